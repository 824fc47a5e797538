// Allocation-free batched solve: vfs_solve_batch with the per-pair solve
// state and the pair descriptors in a fixed device array of the library
// instead of the rig's workspace, for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid it).
#include <mutex>

#include "runtime.h"

using namespace vfs;

namespace {

// Largest state the allocation-free solve holds: descriptors of up to
// kMaxBatch pairs, then the pairs' solve state.
constexpr size_t kScratchBytes = size_t(VFS_NOALLOC_SCRATCH_BYTES);
constexpr size_t kSlotBytes = (sizeof(Slot) * kMaxBatch + 255) / 256 * 256;

// Held by every device the library runs this entry point on, until the
// process ends.  Host code never passes this name to a kernel: it uses the
// device address looked up for the current device (scratch_on_device).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The address of the current device's copy of `scratch`, looked up once per
// device (with that device current).
vfs_status scratch_on_device(char*& out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(VFS_E_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(VFS_E_DEVICE, "device %d beyond the library's table", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VFS_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    out = static_cast<char*>(g_ptr[dev]);
    return VFS_OK;
}

}  // namespace

extern "C" {

vfs_status vfs_solve_batch_noalloc(vfs_rig* r, int n, const float* const* I0, const float* const* I1,
                                   size_t pitch_bytes, float* const* u_out, float* const* w_out,
                                   float* const* depth_out, float* const* z_out, uint8_t* const* valid_out,
                                   const vfs_params* params, const double* betas, const double* etas,
                                   void* hip_stream)
{
    vfs_status st = check_batch(r, n, I0, I1, pitch_bytes, u_out, w_out, depth_out, params, betas, etas, true);
    if (st) return st;
    const PairLayout lay =
        make_layout(r->g, params->storage, params->reg == VFS_TGV, params->data_term != VFS_DATA_BRIGHTNESS);
    const size_t need = kSlotBytes + lay.bytes * size_t(n);
    if (need > kScratchBytes)
        return fail(VFS_E_BUDGET, "%d pair(s) of %dx%d need %zu bytes of state, the allocation-free solve holds %zu",
                    n, r->g.W[0], r->g.H[0], need, kScratchBytes);
    char* base = nullptr;
    st = scratch_on_device(base);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Slot* slots = reinterpret_cast<Slot*>(base);
    // the solve writes every state array before reading it (pyramids, zero
    // state at the coarsest level, transfers, duals reset per level), so the
    // previous call's contents need no clearing
    write_batch_slots(r, n, I0, I1, pitch_bytes, u_out, w_out, depth_out, z_out, valid_out, params, betas, etas,
                      true, base + kSlotBytes, lay, slots, s);
    return solve_slots(slots, n, r->g, *params, s, nullptr);
}

}  // extern "C"
