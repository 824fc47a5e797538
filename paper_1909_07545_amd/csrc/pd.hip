// Primal-dual iteration of the tensor-weighted TGV-L1 energy (Eq. (10)) by
// the Chambolle-Pock scheme of Eq. (11), with the diagonal preconditioning of
// Sec. III-D and the resolvent of Eq. (13).
//
// Iterates: the same sequence as the textbook order
//     y^{k+1} = P(y^k + sigma K xbar^k),  x^{k+1} = prox(x^k - tau K^T y^{k+1}),
//     xbar^{k+1} = x^{k+1} + theta (x^{k+1} - x^k),
// with x = (u, v), y = (p, q), but the state in memory is stored one half
// step apart, (x^{k-1}, y^k).  A PD_FUSED launch computes x^k on the tile plus
// a one-pixel halo, forms xbar^k in registers and finishes with y^{k+1}; xbar
// never touches memory.  A PD_FUSED2 / 3 / 4 launch (pdn_kernel) does N = 2,
// 3 or 4 such iterations in one pass over memory: each trails the one before
// by two rows in the same march, reading its results from registers, so the
// state is read and written once per N iterations.  A warp's K iterations
// (K >= N) are one PD_FIRST2 / 3 / 4 pass (the same pass whose first
// iteration is the dual half alone, y^1 from x^0 = xbar^0), the remaining
// K - N iterations in PD_FUSED / PD_FUSED2 launches and passes of N, and one
// PD_PRIMAL_LAST launch (x^K); with K < N a PD_DUAL_FIRST launch starts it.
// Every launch reads one copy of the state and writes the other.
//
// Storage: p, q and the tensor pack are read and written as FP32, FP16 or
// BF16 (template S); u, v, rho_c and all arithmetic are FP32.
//
// Every launch reads each pair's planes from its slot descriptor; in serving
// ticks the pairs of one launch may be at different levels (the grid covers
// the largest, workgroups beyond a pair's level exit at once).
//
// Work decomposition: one 64-lane wavefront owns a strip of columns (62 for
// the one-iteration modes: lanes 1..62, lanes 0 and 63 are the x-halo;
// 64 - 2N for N iterations) and marches down a
// segment of rows plus a halo above and below, keeping the rows it still
// needs in registers and exchanging x-neighbours by lane shifts.  The four
// wavefronts of a workgroup take four neighbouring strips of the same
// segment, and workgroups are renumbered so that the blocks the dispatcher
// places on one XCD cover a contiguous band of tasks: strips that share
// halo columns are read at the same time through the same L2.  The segment
// height is a run-time argument chosen by the host per launch (march_shape),
// so every grid runs the same code and a pair's result does not depend on
// the batch it is launched with.
#include "vfs_internal.h"

#include <map>
#include <mutex>
#include <utility>

namespace vfs {

// Multiply-adds are fused only within one source expression, never across
// statements, so that code paths which evaluate the same expressions on the
// same values (the two march directions) give bitwise equal results.
#pragma clang fp contract(on)

namespace {

constexpr int kLanes = 64;
constexpr int kWaves = 4;            // wavefronts per workgroup
constexpr int kCols = kLanes - 2;    // owned columns per wavefront, one-iteration modes
// Segment heights (rows per wavefront march).  With enough work for several
// rounds of resident wavefronts: marches of about kBY rows, their count
// rounded to whole rounds (short marches keep the rows in flight at any
// moment close together, measured faster than long ones at equal traffic).
// With less: one round of marches as long as fit, but at least kBYs rows
// (long marches re-read fewer halo rows, and no partly filled last round
// idles the chip); launches too small to fill the SIMDs go shorter
// (short_march_floor).
constexpr int kBY = 16;
// The 16-bit kernels are bound by vector issue rather than by memory: their
// marches aim at 28 rows, which re-compute fewer halo rows (measured on 8
// pairs of 2048x2048, three iterations per pass: 552 us per launch at 16
// rows, 517 at 28, 520 at 36; the FP32 three-iteration pass is slower beyond
// 16: 677, 685 at 22, 693 at 28).
constexpr int kBY16 = 28;
// The FP32 four-iteration kernel spends more vector issue per row than the
// three-iteration one reads bytes: its marches aim at 40 rows (measured on 8
// pairs of 2048x2048 with carried step-size bases, three wavefronts per
// SIMD: 735 us per launch at a 24-row target, 726 at 32, 719 at 40 -- 41-row
// marches in five rounds; without carried bases, four wavefronts per SIMD:
// 817 us at 16, 779 at 24, 770 at 32).  A target that leaves fewer than
// kRoundsForShort rounds falls back to one round of long marches.
constexpr int kBY4 = 40;
constexpr int kBYs = 4;
constexpr long long kRoundsForShort = 4;
constexpr int kXcds = 8;

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// whole-wavefront shifts by one lane (DPP wave_shr:1 / wave_shl:1); the lane
// without a source receives 0 (bound_ctrl: no old value to set up) -- always
// a halo lane whose result is unused
__device__ inline float from_left(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ inline float from_right(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}

struct Row {
    float u;
    float2 v, p;
    float4 q, t;   // t = (t11, t12, t22, I_u)
    float rho;
    unsigned f;
};

__device__ inline Row zero_row()
{
    Row w;
    w.u = 0.f; w.rho = 0.f; w.f = 0u;
    w.v = make_float2(0.f, 0.f);
    w.p = make_float2(0.f, 0.f);
    w.q = make_float4(0.f, 0.f, 0.f, 0.f);
    w.t = make_float4(1.f, 0.f, 1.f, 0.f);
    return w;
}

// One pair's planes at the level of a launch (workgroup-uniform).  State
// pointers already include the level's offset in the level-stacked arrays.
struct Planes {
    int W, H, pitch;
    const float* u_in;
    float* u_out;
    const float2* v_in;
    float2* v_out;
    const void* p_in;
    void* p_out;
    const void* q_in;
    void* q_out;
    const void* tpack;          // single-level
    const float* rho;           // single-level
    const uint8_t* flags;
};

template <int S>
__device__ inline bool planes_of(const PdArgs& a, int z, Planes& P)
{
    Pick pk;
    if (!pick(a.lc, z, pk)) return false;
    const Slot& sl = a.lc.slots[pk.slot];
    const int l = pk.l;
    const long long off = a.lc.g.off[l];
    const int pu = (a.lc.iu ^ int(pk.flip)) & 1, pp = (a.lc.ip ^ int(pk.flip >> 1)) & 1;
    constexpr long long E2 = S == ST_F32 ? 8 : 4, E4 = S == ST_F32 ? 16 : 8;
    P.W = a.lc.g.W[l];
    P.H = a.lc.g.H[l];
    P.pitch = a.lc.g.pitch[l];
    P.u_in = sl.u[pu] + off;
    P.u_out = sl.u[pu ^ 1] + off;
    P.v_in = sl.v[pu] + off;
    P.v_out = sl.v[pu ^ 1] + off;
    P.p_in = static_cast<const char*>(sl.p[pp]) + off * E2;
    P.p_out = static_cast<char*>(sl.p[pp ^ 1]) + off * E2;
    P.q_in = static_cast<const char*>(sl.q[pp]) + off * E4;
    P.q_out = static_cast<char*>(sl.q[pp ^ 1]) + off * E4;
    P.tpack = sl.tpack;
    P.rho = sl.rho;
    P.flags = sl.flags[l];
    return true;
}

// Row reads and writes through buffer resources: one resource per plane row
// (uniform, in scalar registers) and the lane's byte offset in the row (a
// 32-bit vector register, the same at every step), so a row access costs no
// vector address arithmetic.  A resource's record count is the row's width in
// bytes, and the hardware returns zero for a read at or past it and drops
// such a write: a lane left of the image (x < 0 wraps to an offset near 2^32)
// or right of it reads zero, and a row outside the image (or one a march does
// not need) is given a record count of 0 and reads zero -- the zero state of
// the image's surroundings without moves or per-lane branches.  (The tensor
// reads as 0 there, which only ever meets zero mask bits.)  Rows hold far
// fewer than 2^25 columns, so every offset below stays under 2^32.
constexpr int kRsrcWord3 = 0x00020000;   // untyped 32-bit data, no swizzle, no index
// the column offset of a lane that writes nothing: times 4, 8 or 16 bytes it
// is 2^29, 2^30 or 2^31, past any row's records
constexpr uint32_t kNoColumn = 0x08000000u;
// cache policy of a store that the next read will not find in any cache (non-temporal)
constexpr int kStoreNT = 2;

__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const void* plane, long long row, int pitch, int elem, int bytes)
{
    char* base = const_cast<char*>(static_cast<const char*>(plane)) + row * pitch * elem;
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, kRsrcWord3);
}

template <int S> __device__ inline float2 dec2(uint32_t v)
{
    if constexpr (S == ST_F32) return make_float2(0.f, 0.f);
    else return make_float2(dec16<S>(uint16_t(v & 0xffffu)), dec16<S>(uint16_t(v >> 16)));
}

template <int S> __device__ inline float4 dec4(uint32_t lo, uint32_t hi)
{
    if constexpr (S == ST_F32) return make_float4(0.f, 0.f, 0.f, 0.f);
    else return make_float4(dec16<S>(uint16_t(lo & 0xffffu)), dec16<S>(uint16_t(lo >> 16)),
                            dec16<S>(uint16_t(hi & 0xffffu)), dec16<S>(uint16_t(hi >> 16)));
}

template <int S> __device__ inline float2 rd2(__amdgpu_buffer_rsrc_t rs, uint32_t x)
{
    if constexpr (S == ST_F32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, x * 8u, 0, 0);
        return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
    } else {
        return dec2<S>(__builtin_amdgcn_raw_buffer_load_b32(rs, x * 4u, 0, 0));
    }
}

template <int S> __device__ inline float4 rd4(__amdgpu_buffer_rsrc_t rs, uint32_t x)
{
    if constexpr (S == ST_F32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, x * 16u, 0, 0);
        return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, x * 8u, 0, 0);
        return dec4<S>(v[0], v[1]);
    }
}

// Row r of the state planes at every lane (zero outside the image, and for
// rows with valid = false).
template <bool TGV, bool PRIMAL, int S>
__device__ inline Row read_row(const Planes& P, int x, int r, bool valid = true)
{
    constexpr int E2 = S == ST_F32 ? 8 : 4, E4 = S == ST_F32 ? 16 : 8;
    const bool ok = valid && r >= 0 && r < P.H;
    const long long rr = ok ? r : 0;
    const int W = ok ? P.W : 0;
    const uint32_t xo = uint32_t(x);
    Row w;
    w.u = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(row_rsrc(P.u_in, rr, P.pitch, 4, W * 4), xo * 4u, 0, 0));
    w.p = rd2<S>(row_rsrc(P.p_in, rr, P.pitch, E2, W * E2), xo);
    w.t = rd4<S>(row_rsrc(P.tpack, rr, P.pitch, E4, W * E4), xo);
    w.f = __builtin_amdgcn_raw_buffer_load_b8(row_rsrc(P.flags, rr, P.pitch, 1, W), xo, 0, 0);
    w.rho = 0.f;
    if (PRIMAL)
        w.rho = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(row_rsrc(P.rho, rr, P.pitch, 4, W * 4), xo * 4u,
                                                                     0, 0));
    w.v = make_float2(0.f, 0.f);
    w.q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (TGV) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(P.v_in, rr, P.pitch, 8, W * 8), xo * 8u, 0, 0);
        w.v = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
        w.q = rd4<S>(row_rsrc(P.q_in, rr, P.pitch, E4, W * E4), xo);
    }
    return w;
}

// Writes of row r's results by the owner lanes (xs: the lane's column, or
// a column past any row for the other lanes); with NT non-temporally.
template <int POLICY>
__device__ inline void store_b32(uint32_t v, __amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, off, 0, POLICY);
}
template <int POLICY>
__device__ inline void store_b64(__attribute__((ext_vector_type(2))) uint32_t v, __amdgpu_buffer_rsrc_t rs,
                                 uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, off, 0, POLICY);
}
template <int POLICY>
__device__ inline void store_b128(__attribute__((ext_vector_type(4))) uint32_t v, __amdgpu_buffer_rsrc_t rs,
                                  uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, POLICY);
}

template <bool TGV, int POLICY>
__device__ inline void write_primal_p(const Planes& P, uint32_t xs, int r, float un, float2 vn)
{
    store_b32<POLICY>(__float_as_uint(un), row_rsrc(P.u_out, r, P.pitch, 4, P.W * 4), xs * 4u);
    if (TGV) {
        const __attribute__((ext_vector_type(2))) uint32_t v = {__float_as_uint(vn.x), __float_as_uint(vn.y)};
        store_b64<POLICY>(v, row_rsrc(P.v_out, r, P.pitch, 8, P.W * 8), xs * 8u);
    }
}

template <bool TGV, int S, int POLICY>
__device__ inline void write_dual_p(const Planes& P, uint32_t xs, int r, float2 pn, float4 qn)
{
    if constexpr (S == ST_F32) {
        const __attribute__((ext_vector_type(2))) uint32_t pv = {__float_as_uint(pn.x), __float_as_uint(pn.y)};
        store_b64<POLICY>(pv, row_rsrc(P.p_out, r, P.pitch, 8, P.W * 8), xs * 8u);
        if (TGV) {
            const __attribute__((ext_vector_type(4))) uint32_t qv = {__float_as_uint(qn.x), __float_as_uint(qn.y),
                                                                     __float_as_uint(qn.z), __float_as_uint(qn.w)};
            store_b128<POLICY>(qv, row_rsrc(P.q_out, r, P.pitch, 16, P.W * 16), xs * 16u);
        }
    } else {
        const uint32_t pv = uint32_t(enc16<S>(pn.x)) | (uint32_t(enc16<S>(pn.y)) << 16);
        store_b32<POLICY>(pv, row_rsrc(P.p_out, r, P.pitch, 4, P.W * 4), xs * 4u);
        if (TGV) {
            const __attribute__((ext_vector_type(2))) uint32_t qv = {
                uint32_t(enc16<S>(qn.x)) | (uint32_t(enc16<S>(qn.y)) << 16),
                uint32_t(enc16<S>(qn.z)) | (uint32_t(enc16<S>(qn.w)) << 16)};
            store_b64<POLICY>(qv, row_rsrc(P.q_out, r, P.pitch, 8, P.W * 8), xs * 8u);
        }
    }
}

template <bool TGV>
__device__ inline void write_primal(const Planes& P, uint32_t xs, int r, float un, float2 vn, bool nt = false)
{
    if (nt) write_primal_p<TGV, kStoreNT>(P, xs, r, un, vn);
    else write_primal_p<TGV, 0>(P, xs, r, un, vn);
}

template <bool TGV, int S>
__device__ inline void write_dual(const Planes& P, uint32_t xs, int r, float2 pn, float4 qn, bool nt = false)
{
    if (nt) write_dual_p<TGV, S, kStoreNT>(P, xs, r, pn, qn);
    else write_dual_p<TGV, S, 0>(P, xs, r, pn, qn);
}

// A flag bit as the float 0 or 1 that multiplies a masked difference: a
// bit-field extract and one conversion.
template <unsigned B>
__device__ inline float flag_bit(unsigned f)
{
    static_assert(B && !(B & (B - 1)), "one flag bit");
    return float((f >> __builtin_ctz(B)) & 1u);
}

// What the primal step of row r reads from row r - 1 (the y-parts of the
// masked divergences and of the column sums of the preconditioner).
struct Above {
    float b, cy, my, myq2, myq4;
};

// The parts of a row's "above" contribution that the step sizes need (they
// depend on the tensor and the mask bits only).
__device__ inline void above_steps(float4 t, unsigned f, float& cy, float& my)
{
    my = flag_bit<F_MY>(f);
    cy = my * (fabsf(t.y) + fabsf(t.z));
}

__device__ inline Above above_of(float2 p, float4 q, float4 t, unsigned f)
{
    Above ab;
    float my;
    above_steps(t, f, ab.cy, my);
    ab.b = my * (t.y * p.x + t.z * p.y);
    ab.my = my;
    ab.myq2 = my * q.y;
    ab.myq4 = my * q.w;
    return ab;
}

// Resolvent of the linearised data term, Eq. (13) (third case with the sign
// that zeroes rho_bar = rho_c + u I_u).
__device__ inline float resolvent(float uhat, float rho, float Iu, float tau, float lambda)
{
    const float rb = rho + uhat * Iu;
    const float a = tau * lambda * Iu;
    const float aI = a * Iu;
    if (rb < -aI) return uhat + a;
    if (rb > aI) return uhat - a;
    if (Iu == 0.f) return uhat;
    return uhat - rb * frcp(Iu);
}

// Step sizes of the diagonal preconditioning (Sec. III-D) at a pixel, before
// an iteration's schedule factor: the primal steps of u and v from the
// pixel's tensor and mask bits, its left neighbour's (lane shifts; every lane
// of the wavefront calls this) and the row above's (cy, my of above_steps).
struct PrimalBases {
    float tu, tv;
};

template <bool TGV>
__device__ inline PrimalBases primal_bases(float4 t, unsigned f, float cy_up, float my_up, float a0, float a1)
{
    const float mx = flag_bit<F_MX>(f);
    const float my = flag_bit<F_MY>(f);
    const float cx = mx * (fabsf(t.x) + fabsf(t.y));
    const float cx_l = from_left(cx);
    const float cu = fabsf(t.x * mx + t.y * my) + fabsf(t.y * mx + t.z * my) + cx_l + cy_up;
    PrimalBases b;
    b.tu = cu > 0.f ? frcp(a1 * cu) : frcp(a1);
    b.tv = 0.f;
    if (TGV) {
        const float mx_l = from_left(mx);
        b.tv = frcp(a1 + a0 * (mx + my + mx_l + my_up));
    }
    return b;
}

// The dual step of p at a pixel, before an iteration's schedule factor.
template <bool TGV>
__device__ inline float dual_base(float4 t, unsigned f, float a1)
{
    const float pmx = flag_bit<F_MX>(f);
    const float pmy = flag_bit<F_MY>(f);
    const float vrow = TGV ? a1 : 0.f;
    const float s1 = a1 * (fabsf(t.x * pmx + t.y * pmy) + fabsf(t.x) * pmx + fabsf(t.y) * pmy) + vrow;
    const float s2 = a1 * (fabsf(t.y * pmx + t.z * pmy) + fabsf(t.y) * pmx + fabsf(t.z) * pmy) + vrow;
    const float smax = fmaxf(s1, s2);
    return smax > 0.f ? frcp(smax) : frcp(a1);
}

// Primal step at one pixel: x^k from x^{k-1} = (u, v) and y^k = (p, q) at the
// pixel, its left neighbour (lane shifts) and the row above (ab), with the
// steps tau_u, tau_v (bases times the iteration's factor).  Called by every
// lane of the wavefront (it shifts across lanes).  Returns (un, vn); the pixel
// is left unchanged outside the mask.
template <bool TGV>
__device__ inline void primal_step(float u, float2 v, float2 p, float4 q, float4 t, float rho, unsigned f,
                                   const Above& ab, float a0, float a1, float lambda, float tau_u, float tau_v,
                                   float& un, float2& vn)
{
    const float mx = flag_bit<F_MX>(f);
    const float my = flag_bit<F_MY>(f);
    const float ax = mx * (t.x * p.x + t.y * p.y);
    const float ax_l = from_left(ax);
    const float b = my * (t.y * p.x + t.z * p.y);
    const float divtp = ax - ax_l + b - ab.b;
    const float ur = resolvent(u + tau_u * a1 * divtp, rho, t.w, tau_u, lambda);
    float2 vr = v;
    if (TGV) {
        const float mxq1 = mx * q.x, mxq3 = mx * q.z;
        const float mxq1_l = from_left(mxq1), mxq3_l = from_left(mxq3);
        const float d1 = mxq1 - mxq1_l + my * q.y - ab.myq2;
        const float d2 = mxq3 - mxq3_l + my * q.w - ab.myq4;
        vr.x = v.x + tau_v * (a1 * p.x + a0 * d1);
        vr.y = v.y + tau_v * (a1 * p.y + a0 * d2);
    }
    const bool msk = (f & F_MASK) != 0u;
    un = msk ? ur : u;
    vn = msk ? vr : v;
}

// Dual step at one pixel of row s: y^{k+1} from y^k = (p, q) and xbar^k at
// the pixel (ub, vb), its right neighbour (ub_r, vb_r; shifted by the caller)
// and the row below (ub_d, vb_d).  sig is the step of p (base times the
// iteration's factor); sq is the step of q, ss / (2 alpha0), computed once per
// march by the caller.  The duals stay as they are outside the mask.
template <bool TGV>
__device__ inline void dual_step(float2 p, float4 q, float4 t, unsigned f, float ub, float2 vb, float ub_r,
                                 float2 vb_r, float ub_d, float2 vb_d, float a0, float a1, float sig, float sq,
                                 float2& pn, float4& qn)
{
    pn = p;
    qn = q;
    if (!(f & F_MASK)) return;
    const float pmx = flag_bit<F_MX>(f);
    const float pmy = flag_bit<F_MY>(f);
    const float gx = pmx * (ub_r - ub), gy = pmy * (ub_d - ub);
    float p1 = p.x + sig * a1 * (t.x * gx + t.y * gy - (TGV ? vb.x : 0.f));
    float p2 = p.y + sig * a1 * (t.y * gx + t.z * gy - (TGV ? vb.y : 0.f));
    const float n2 = p1 * p1 + p2 * p2;
    if (n2 > 1.f) {
        const float inv = __builtin_amdgcn_rsqf(n2);
        p1 *= inv;
        p2 *= inv;
    }
    pn = make_float2(p1, p2);
    if (TGV) {
        float q1 = q.x + sq * a0 * pmx * (vb_r.x - vb.x);
        float q2 = q.y + sq * a0 * pmy * (vb_d.x - vb.x);
        float q3 = q.z + sq * a0 * pmx * (vb_r.y - vb.y);
        float q4 = q.w + sq * a0 * pmy * (vb_d.y - vb.y);
        const float m2 = q1 * q1 + q2 * q2 + q3 * q3 + q4 * q4;
        if (m2 > 1.f) {
            const float inv = __builtin_amdgcn_rsqf(m2);
            q1 *= inv; q2 *= inv; q3 *= inv; q4 *= inv;
        }
        qn = make_float4(q1, q2, q3, q4);
    }
}

// The steps above with the step sizes computed at the point of use: ts and ss
// are the iteration's factors of the primal and dual steps.
template <bool TGV>
__device__ inline void primal_at(float u, float2 v, float2 p, float4 q, float4 t, float rho, unsigned f,
                                 const Above& ab, float a0, float a1, float lambda, float ts, float& un, float2& vn)
{
    const PrimalBases b = primal_bases<TGV>(t, f, ab.cy, ab.my, a0, a1);
    primal_step<TGV>(u, v, p, q, t, rho, f, ab, a0, a1, lambda, b.tu * ts, b.tv * ts, un, vn);
}

template <bool TGV>
__device__ inline void dual_at(float2 p, float4 q, float4 t, unsigned f, float ub, float2 vb, float ub_r,
                               float2 vb_r, float ub_d, float2 vb_d, float a0, float a1, float ss, float sq,
                               float2& pn, float4& qn)
{
    dual_step<TGV>(p, q, t, f, ub, vb, ub_r, vb_r, ub_d, vb_d, a0, a1, dual_base<TGV>(t, f, a1) * ss, sq, pn, qn);
}

// XCD-aware renumbering of the workgroup index.
__device__ inline int logical_block()
{
    const int nb = gridDim.x, bid = blockIdx.x;
    const int xcd = bid % kXcds, k = bid / kXcds, qn = nb / kXcds, rn = nb % kXcds;
    return xcd < rn ? xcd * (qn + 1) + k : rn * (qn + 1) + (xcd - rn) * qn + k;
}

// The march of this wavefront: strip tx of `cols` columns and rows from y0 of
// pair `pair`; false if the grid's last workgroup has no task for it.
struct Task {
    int tx, y0, pair;
};

__device__ inline bool task_of(const PdArgs& a, int cols, int by, int segs, Task& t)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const long long task = (long long)logical_block() * kWaves + wave;
    const int tiles_x = (a.lc.g.W[a.lc.gl] + cols - 1) / cols;
    const long long pair = task / ((long long)tiles_x * segs);
    t.tx = int(task % tiles_x);
    t.y0 = int((task / tiles_x) % segs) * by;
    t.pair = int(pair);
    return pair < a.lc.n;
}

// One iteration (PD_FUSED) or its first / last half (PD_DUAL_FIRST, PD_PRIMAL_LAST).
template <int MODE, bool TGV, int S>
__global__ __launch_bounds__(kLanes * kWaves) void pd_kernel(PdArgs a, int by, int segs)
{
    constexpr bool PRIMAL = MODE != PD_DUAL_FIRST;
    constexpr bool DUAL = MODE != PD_PRIMAL_LAST;

    Task tk;
    if (!task_of(a, kCols, by, segs, tk)) return;
    Planes P;
    if (!planes_of<S>(a, tk.pair, P)) return;
    const int tx = tk.tx;
    if (tx * kCols >= P.W) return;

    const int lane = threadIdx.x & (kLanes - 1);
    const int x = tx * kCols - 1 + lane;
    const bool owner = lane >= 1 && lane <= kCols && x < P.W;
    const uint32_t xs = owner ? uint32_t(x) : kNoColumn;
    const int y0 = tk.y0;
    if (y0 >= P.H) return;
    const int y1 = min(y0 + by, P.H);           // owned rows [y0, y1)
    const float a0 = a.alpha0, a1 = a.alpha1;
    const float sq1 = a.sigma_scale / (2.f * a0);   // the step of q, once per march

    // row r - 1 as the dual step needs it
    float2 p_prev = make_float2(0.f, 0.f);
    float4 q_prev = make_float4(0.f, 0.f, 0.f, 0.f), t_prev = make_float4(1.f, 0.f, 1.f, 0.f);
    unsigned f_prev = 0u;
    float ub_prev = 0.f;
    float2 vb_prev = make_float2(0.f, 0.f);
    Above ab = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (PRIMAL) {
        const Row w = read_row<TGV, false, S>(P, x, y0 - 1);
        ab = above_of(w.p, w.q, w.t, w.f);
    }

    const int r_end = DUAL ? y1 : y1 - 1;       // last row visited (row y1 is the look-ahead)
    // rows are loaded one step ahead of their use, so that a row's memory
    // latency overlaps the previous row's arithmetic (the multi-iteration
    // kernels weigh this against occupancy, see below)
    constexpr bool PF = true;
    Row nxt = zero_row();
    if constexpr (PF) nxt = read_row<TGV, PRIMAL, S>(P, x, y0);
    for (int r = y0; r <= r_end; ++r) {
        Row c;
        if constexpr (PF) {
            c = nxt;
            if (r + 1 <= r_end) nxt = read_row<TGV, PRIMAL, S>(P, x, r + 1);
        } else {
            c = read_row<TGV, PRIMAL, S>(P, x, r);
        }
        // primal step at row r: x^k from x^{k-1} and y^k
        float un = c.u;
        float2 vn = c.v;
        if (PRIMAL) {
            primal_at<TGV>(c.u, c.v, c.p, c.q, c.t, c.rho, c.f, ab, a0, a1, a.lambda, a.tau_scale, un, vn);
            if (r < y1) write_primal<TGV>(P, xs, r, un, vn);
        }
        // over-relaxation (xbar stays in registers)
        const float ub = un + a.theta * (un - c.u);
        const float2 vb = make_float2(vn.x + a.theta * (vn.x - c.v.x), vn.y + a.theta * (vn.y - c.v.y));
        // dual step at row r - 1: y^{k+1} from y^k and xbar^k
        if (DUAL) {
            const float ub_r = from_right(ub_prev);
            const float2 vb_r = make_float2(from_right(vb_prev.x), from_right(vb_prev.y));
            if (r > y0) {
                float2 pn;
                float4 qn;
                dual_at<TGV>(p_prev, q_prev, t_prev, f_prev, ub_prev, vb_prev, ub_r, vb_r, ub, vb, a0, a1,
                             a.sigma_scale, sq1, pn, qn);
                write_dual<TGV, S>(P, xs, r - 1, pn, qn);
            }
        }
        // slide the window
        p_prev = c.p;
        q_prev = c.q;
        t_prev = c.t;
        f_prev = c.f;
        ub_prev = ub;
        vb_prev = vb;
        ab = above_of(c.p, c.q, c.t, c.f);
    }
}

// N iterations per pass: (x^{k-1}, y^k) -> (x^{k+N-1}, y^{k+N}).  At march
// step r, iteration i (0-based)
// takes its primal step at row r - 2i and its dual step at row r - 2i - 1.
// Iteration i's primal step reads x^{k+i-1} from iteration i-1's primal step
// two steps earlier, y^{k+i} from iteration i-1's dual step one step earlier
// (and two steps earlier for the row above); its dual step reads its own
// xbar of the previous and the current step.  Iteration i covers rows
// [y0 - (N-1-i), y1 + (N-1-i)] (primal) and one row fewer below (dual), so
// the last iteration produces exactly the owned rows [y0, y1).  Column
// validity shrinks by one lane per iteration on each side: the wavefront
// owns lanes N .. 63-N.  The row constants (tensor, rho_c, flags) of the
// last 2N rows stay in registers (or in LDS, RowConsts).
// The tensor pack as kept in a register delay line: FP32 as is, the 16-bit
// modes packed (as stored) and decoded at each use.
template <int S> struct TensorRaw {
    using type = uint2;
    __device__ static uint2 pack(float4 t)
    {
        return make_uint2(uint32_t(enc16<S>(t.x)) | (uint32_t(enc16<S>(t.y)) << 16),
                          uint32_t(enc16<S>(t.z)) | (uint32_t(enc16<S>(t.w)) << 16));
    }
    __device__ static float4 unpack(uint2 v)
    {
        return make_float4(dec16<S>(uint16_t(v.x & 0xffffu)), dec16<S>(uint16_t(v.x >> 16)),
                           dec16<S>(uint16_t(v.y & 0xffffu)), dec16<S>(uint16_t(v.y >> 16)));
    }
    __device__ static uint2 identity() { return pack(make_float4(1.f, 0.f, 1.f, 0.f)); }
};
template <> struct TensorRaw<ST_F32> {
    using type = float4;
    __device__ static float4 pack(float4 t) { return t; }
    __device__ static float4 unpack(float4 t) { return t; }
    __device__ static float4 identity() { return make_float4(1.f, 0.f, 1.f, 0.f); }
};

// The row constants (tensor pack as stored, rho_c) of the last D rows of a
// march: a register delay line shifted at every step, or a ring in LDS, one
// per wavefront, where the row entering at a step takes slot h, the row that
// entered d steps earlier sits at slot (h + d) mod D and h steps back by one
// per step.  The ring holds the four-iteration kernels' rows out of the
// registers (40 KB of LDS per workgroup): with it and the carried step-size
// bases they take 150 VGPRs in FP32, three wavefronts per SIMD; with the rows
// in registers as well they would drop to two.  The three-iteration kernels
// keep their six rows in registers: the ring saves them no wavefront and its
// index arithmetic costs as much as the moves it saves (measured: equal
// times).
template <typename TRaw, int D, bool RING> struct RowConsts {
    TRaw t[D];
    float rho[D];
    __device__ void init(TRaw id)
    {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            t[d] = id;
            rho[d] = 0.f;
        }
    }
    __device__ void set_first(TRaw v) { t[0] = v; }
    __device__ void push(TRaw v, float r)
    {
#pragma unroll
        for (int d = D - 1; d > 0; --d) {
            t[d] = t[d - 1];
            rho[d] = rho[d - 1];
        }
        t[0] = v;
        rho[0] = r;
    }
    __device__ TRaw tens(int d) const { return t[d]; }
    __device__ float rh(int d) const { return rho[d]; }
};

template <typename TRaw, int D> struct RowConsts<TRaw, D, true> {
    TRaw (*t)[kLanes];     // this wavefront's D slots of 64 lanes in LDS
    float (*rho)[kLanes];
    int h, ln;
    __device__ int at(int d) const
    {
        const int k = h + d;
        return k >= D ? k - D : k;
    }
    __device__ void init(TRaw id)
    {
        h = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            t[d][ln] = id;
            rho[d][ln] = 0.f;
        }
    }
    __device__ void set_first(TRaw v) { t[h][ln] = v; }
    __device__ void push(TRaw v, float r)
    {
        h = h == 0 ? D - 1 : h - 1;
        t[h][ln] = v;
        rho[h][ln] = r;
    }
    __device__ TRaw tens(int d) const { return t[at(d)][ln]; }
    __device__ float rh(int d) const { return rho[at(d)][ln]; }
};

// Whether a march computes each row's step-size bases once, when the row
// enters, and carries them in a delay line beside the tensor, or at every use.
// Both give the same values.  Carried in the TGV kernels of three and four
// iterations: the three-iteration kernels keep four wavefronts per SIMD with
// them (FP32 133 VGPRs is the exception, three), the four-iteration ones drop
// to three (150 VGPRs in FP32) and are still faster: their marches issue 12 to
// 15 % fewer vector instructions (measured on 8 pairs of 2048x2048: 738 ->
// 726 us per launch at the same march height).
template <bool TGV, int S, int N> constexpr bool kCarryBases = TGV && N >= 2;

// A step's parity as a type: the marches run two steps per loop trip, so
// that the slot of a two-step window that a step reads or writes is a
// constant and the windows slide without register moves.
template <int V> struct Par {
    static constexpr int v = V;
};

// Downward march: at step r, iteration i takes its primal step at row r - 2i
// and its dual step at row r - 2i - 1 (the dual needs xbar of the row below).
template <bool TGV, int S, int N, bool FIRST>
__device__ __forceinline__ void march_down(const PdArgs& a, const Planes& P, int x, bool owner, int y0, int y1,
                                           typename TensorRaw<S>::type (*ringT)[kLanes], float (*ringR)[kLanes])
{
    constexpr int D = 2 * N;    // depth of the constants' delay line
    const float a0 = a.alpha0, a1 = a.alpha1, lam = a.lambda;
    float sqn[N];   // the steps of q, once per march
#pragma unroll
    for (int i = 0; i < N; ++i) sqn[i] = a.sigma_n[i] / (2.f * a0);

    // constants of rows r - d (d = 0 .. D-1) after the shift of step r: the
    // tensor pack as stored (16-bit modes keep it packed until use), rho_c,
    // and the flag bytes packed 8 bits per row into one 64-bit shift register
    using TRaw = typename TensorRaw<S>::type;
    constexpr bool RING = N >= 4;
    RowConsts<TRaw, D, RING> K;
    if constexpr (RING) {
        K.t = ringT;
        K.rho = ringR;
        K.ln = int(threadIdx.x) & (kLanes - 1);
    }
    K.init(TensorRaw<S>::identity());
    uint64_t fD = 0;
    auto flag = [&](int d) { return unsigned(fD >> (8 * d)) & 0xffu; };
    // carried step-size bases of rows r - d (primal of u and v, dual of p),
    // and the step-size part of the row above the entering row
    constexpr bool CB = kCarryBases<TGV, S, N>;
    float tuD[D], tvD[D], sgD[D];
    float cy_up = 0.f, my_up = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) tuD[d] = tvD[d] = sgD[d] = 0.f;
    // per iteration i: its primal outputs x and dual outputs y of the last
    // two steps, in slots by the parity of the step that wrote them (a step
    // of parity s finds the previous step's values in slot s ^ 1 and the
    // ones before in slot s, then writes slot s), and its xbar of the last
    // step
    float xu[N][2], xbu[N];
    float2 xv[N][2], xbv[N], yp[N][2];
    float4 yq[N][2];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xbu[i] = 0.f;
        xbv[i] = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            xu[i][k] = 0.f;
            xv[i][k] = make_float2(0.f, 0.f);
            yp[i][k] = make_float2(0.f, 0.f);
            yq[i][k] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    // y^k of the rows of the last two steps (from memory) for iteration 0, in
    // the same slots; the row above the first step (which has parity 0)
    float2 pm[2];
    float4 qm[2];
    pm[0] = make_float2(0.f, 0.f);
    qm[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    {
        const Row w = read_row<TGV, false, S>(P, x, y0 - N);
        pm[1] = w.p;
        qm[1] = w.q;
        K.set_first(TensorRaw<S>::pack(w.t));
        fD = w.f;
        above_steps(w.t, w.f, cy_up, my_up);
    }
    const int r_lo = y0 - (N - 1), r_hi = y1 + 2 * N - 2, r_load = y1 + N - 1;
    const uint32_t xs = owner ? uint32_t(x) : kNoColumn;
    const bool nt = S == ST_F32 && a.nt_stores;
    // PF: the next step's row is read one step ahead, into the other slot,
    // where the registers allow it without losing a wavefront per SIMD: the
    // four-iteration kernels (168 VGPRs in FP32, three wavefronts per SIMD;
    // measured on 8 pairs of 2048x2048: 720 -> 706 us per launch with the
    // prefetch in both marches) and the FP32 three-iteration kernel, which
    // runs three wavefronts per SIMD without it too (133 -> 150 VGPRs; whole
    // solves of a 1280x1024 pair 55.7 -> 58.3 Gpix-iter/s, 640x480 19.6 ->
    // 20.8).  The 16-bit three-iteration kernel would drop to three.
    constexpr bool PF = N >= 4 || (N == 3 && S == ST_F32);
    Row rw[2];
    if constexpr (PF) {
        rw[0] = read_row<TGV, true, S>(P, x, r_lo);
        rw[1] = zero_row();
    }
    auto step = [&](const int r, auto par) {
        constexpr int s = decltype(par)::v, o = s ^ 1;
        if constexpr (PF) rw[o] = read_row<TGV, true, S>(P, x, r + 1, r + 1 <= r_load);
        else rw[s] = read_row<TGV, true, S>(P, x, r, r <= r_load);
        const Row& c = rw[s];
        K.push(TensorRaw<S>::pack(c.t), c.rho);
        fD = (fD << 8) | c.f;
        if constexpr (CB) {
#pragma unroll
            for (int d = D - 1; d > 0; --d) {
                tuD[d] = tuD[d - 1];
                tvD[d] = tvD[d - 1];
                sgD[d] = sgD[d - 1];
            }
            const PrimalBases b = primal_bases<TGV>(c.t, c.f, cy_up, my_up, a0, a1);
            tuD[0] = b.tu;
            tvD[0] = b.tv;
            sgD[0] = dual_base<TGV>(c.t, c.f, a1);
            above_steps(c.t, c.f, cy_up, my_up);
        }

        // Later iterations first: iteration i reads iteration i - 1's
        // windows as they stood after the previous step.  An iteration
        // writes its windows only at steps inside its rows; it is inside
        // them at the two steps before any step at which iteration i + 1
        // (or its own dual) reads them, so every read sees the value of the
        // step it means.
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int i = N - 1 - k;
            const int lo = y0 - (N - 1 - i), hi = y1 + (N - 1 - i);
            // primal step of iteration i at row r - 2i
            const int pr = r - 2 * i;
            if (pr < lo || pr > hi) continue;
            const float u_in = i == 0 ? c.u : xu[i - 1][s];
            const float2 v_in = i == 0 ? c.v : xv[i - 1][s];
            const float2 p_in = i == 0 ? c.p : yp[i - 1][o];
            const float4 q_in = i == 0 ? c.q : yq[i - 1][o];
            const float4 t_ab = TensorRaw<S>::unpack(K.tens(2 * i + 1));
            const Above ab = i == 0 ? above_of(pm[o], qm[o], t_ab, flag(1))
                                    : above_of(yp[i - 1][s], yq[i - 1][s], t_ab, flag(2 * i + 1));
            float un = u_in;
            float2 vn = v_in;
            const float4 t_q = i == 0 ? c.t : TensorRaw<S>::unpack(K.tens(2 * i));
            const float rho_q = i == 0 ? c.rho : K.rh(2 * i);
            if (FIRST && i == 0) {
                // the first half iteration: no primal step (xbar^0 = x^0)
            } else if constexpr (CB) {
                primal_step<TGV>(u_in, v_in, p_in, q_in, t_q, rho_q, flag(2 * i), ab, a0, a1, lam,
                                 tuD[2 * i] * a.tau_n[i], tvD[2 * i] * a.tau_n[i], un, vn);
            } else {
                primal_at<TGV>(u_in, v_in, p_in, q_in, t_q, rho_q, flag(2 * i), ab, a0, a1, lam, a.tau_n[i],
                               un, vn);
            }
            const float th = a.theta_n[i];
            const float ubn = un + th * (un - u_in);
            const float2 vbn = make_float2(vn.x + th * (vn.x - v_in.x), vn.y + th * (vn.y - v_in.y));
            if (i == N - 1 && pr >= y0 && pr < y1) write_primal<TGV>(P, xs, pr, un, vn, nt);
            // dual step of iteration i at row r - 2i - 1 (inside its rows
            // whenever the row below is, save the first)
            const int dr = pr - 1;
            if (dr >= lo) {
                const float2 py = i == 0 ? pm[o] : yp[i - 1][s];
                const float4 qy = i == 0 ? qm[o] : yq[i - 1][s];
                const float ub_r = from_right(xbu[i]);
                const float2 vb_r = make_float2(from_right(xbv[i].x), from_right(xbv[i].y));
                float2 pn;
                float4 qn;
                if constexpr (CB)
                    dual_step<TGV>(py, qy, t_ab, flag(2 * i + 1), xbu[i], xbv[i], ub_r, vb_r, ubn, vbn, a0, a1,
                                   sgD[2 * i + 1] * a.sigma_n[i], sqn[i], pn, qn);
                else
                    dual_at<TGV>(py, qy, t_ab, flag(2 * i + 1), xbu[i], xbv[i], ub_r, vb_r, ubn, vbn, a0, a1,
                                 a.sigma_n[i], sqn[i], pn, qn);
                if (i == N - 1 && dr >= y0 && dr < y1) write_dual<TGV, S>(P, xs, dr, pn, qn, nt);
                yp[i][s] = pn;
                yq[i][s] = qn;
            }
            xu[i][s] = un;
            xv[i][s] = vn;
            xbu[i] = ubn;
            xbv[i] = vbn;
        }
        pm[s] = c.p;
        qm[s] = c.q;
    };
    for (int r = r_lo; r <= r_hi; r += 2) {
        step(r, Par<0>());
        if (r + 1 <= r_hi) step(r + 1, Par<1>());
    }
}

// Upward march: at step r (rows decreasing), iteration i takes both its
// primal and its dual step at row r + i.  The primal step needs the duals of
// the row above, which iteration i - 1 produced earlier in the same step; the
// dual step needs xbar of the row below, from iteration i's previous step.
// Iteration i covers the same rows as in the downward march, so every value
// is computed from the same inputs.
template <bool TGV, int S, int N, bool FIRST>
__device__ __forceinline__ void march_up(const PdArgs& a, const Planes& P, int x, bool owner, int y0, int y1,
                                         typename TensorRaw<S>::type (*ringT)[kLanes], float (*ringR)[kLanes])
{
    const float a0 = a.alpha0, a1 = a.alpha1, lam = a.lambda;
    float sqn[N];   // the steps of q, once per march
#pragma unroll
    for (int i = 0; i < N; ++i) sqn[i] = a.sigma_n[i] / (2.f * a0);
    // constants of rows r + d (d = 0 .. N-1) after the push of step r (in
    // the four-iteration kernels: N slots of the LDS ring of march_down)
    using TRaw = typename TensorRaw<S>::type;
    constexpr bool RING = N >= 4;
    RowConsts<TRaw, N, RING> K;
    if constexpr (RING) {
        K.t = ringT;
        K.rho = ringR;
        K.ln = int(threadIdx.x) & (kLanes - 1);
    }
    K.init(TensorRaw<S>::identity());
    uint64_t fD = 0;
    auto flag = [&](int d) { return unsigned(fD >> (8 * d)) & 0xffu; };
    // carried step-size bases of rows r + d (primal of u and v, dual of p)
    constexpr bool CB = kCarryBases<TGV, S, N>;
    float tuD[N], tvD[N], sgD[N];
#pragma unroll
    for (int d = 0; d < N; ++d) tuD[d] = tvD[d] = sgD[d] = 0.f;
    // per iteration i: primal output, xbar and dual output of the previous
    // step (row r + 1 + i) in slot s ^ 1 and of the current step in slot s
    float xu[N][2], xbu[N][2];
    float2 xv[N][2], xbv[N][2], yp[N][2];
    float4 yq[N][2];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            xu[i][k] = 0.f;
            xbu[i][k] = 0.f;
            xv[i][k] = make_float2(0.f, 0.f);
            xbv[i][k] = make_float2(0.f, 0.f);
            yp[i][k] = make_float2(0.f, 0.f);
            yq[i][k] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    const int r_hi = y1 + N - 1, r_lo = y0 - (N - 1);
    const uint32_t xs = owner ? uint32_t(x) : kNoColumn;
    const bool nt = S == ST_F32 && a.nt_stores;
    // the current row and the row above it, in slots as above: the row above
    // of one step is the current row of the next
    Row rw[2];
    rw[0] = zero_row();
    rw[1] = read_row<TGV, true, S>(P, x, r_hi);
    // PFU: the row above the next step's row is read one step ahead too (in
    // the kernels that prefetch in march_down)
    constexpr bool PFU = N >= 4 || (N == 3 && S == ST_F32);
    Row pf;
    if constexpr (PFU) pf = read_row<TGV, true, S>(P, x, r_hi - 1);
    auto step = [&](const int r, auto par) {
        constexpr int s = decltype(par)::v, o = s ^ 1;
        // the row above: iteration 0's y^k there, and the next step's row
        if constexpr (PFU) {
            rw[s] = pf;
            pf = read_row<TGV, true, S>(P, x, r - 2, r - 2 >= r_lo - 1);
        } else {
            rw[s] = read_row<TGV, true, S>(P, x, r - 1);
        }
        const Row& c = rw[o];
        const Row& nx = rw[s];
        K.push(TensorRaw<S>::pack(c.t), c.rho);
        fD = (fD << 8) | c.f;
        if constexpr (CB) {
#pragma unroll
            for (int d = N - 1; d > 0; --d) {
                tuD[d] = tuD[d - 1];
                tvD[d] = tvD[d - 1];
                sgD[d] = sgD[d - 1];
            }
            float cy_up, my_up;
            above_steps(nx.t, nx.f, cy_up, my_up);
            const PrimalBases b = primal_bases<TGV>(c.t, c.f, cy_up, my_up, a0, a1);
            tuD[0] = b.tu;
            tvD[0] = b.tv;
            sgD[0] = dual_base<TGV>(c.t, c.f, a1);
        }

#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int lo = y0 - (N - 1 - i), hi = y1 + (N - 1 - i);
            const int q = r + i;
            const float u_in = i == 0 ? c.u : xu[i - 1][o];
            const float2 v_in = i == 0 ? c.v : xv[i - 1][o];
            const float2 p_in = i == 0 ? c.p : yp[i - 1][o];
            const float4 q_in = i == 0 ? c.q : yq[i - 1][o];
            const float4 t_q = i == 0 ? c.t : TensorRaw<S>::unpack(K.tens(i));
            const float rho_q = i == 0 ? c.rho : K.rh(i);
            // every slot s is written at every step (zero outside the
            // iteration's rows), so what a step leaves in slot s ^ 1 is dead
            // once the step has read it
            float un = 0.f, ub = 0.f;
            float2 vn = make_float2(0.f, 0.f), vb = make_float2(0.f, 0.f);
            if (q >= lo && q <= hi) {
                const Above ab = i == 0 ? above_of(nx.p, nx.q, nx.t, nx.f)
                                        : above_of(yp[i - 1][s], yq[i - 1][s],
                                                   i == 1 ? c.t : TensorRaw<S>::unpack(K.tens(i - 1)), flag(i - 1));
                if (FIRST && i == 0) {
                    // the first half iteration: no primal step (xbar^0 = x^0)
                    un = u_in;
                    vn = v_in;
                } else if constexpr (CB) {
                    primal_step<TGV>(u_in, v_in, p_in, q_in, t_q, rho_q, flag(i), ab, a0, a1, lam, tuD[i] * a.tau_n[i],
                                     tvD[i] * a.tau_n[i], un, vn);
                } else {
                    primal_at<TGV>(u_in, v_in, p_in, q_in, t_q, rho_q, flag(i), ab, a0, a1, lam, a.tau_n[i], un, vn);
                }
                const float th = a.theta_n[i];
                ub = un + th * (un - u_in);
                vb = make_float2(vn.x + th * (vn.x - v_in.x), vn.y + th * (vn.y - v_in.y));
                if (i == N - 1 && q >= y0 && q < y1) write_primal<TGV>(P, xs, q, un, vn, nt);
            }
            xu[i][s] = un;
            xv[i][s] = vn;
            xbu[i][s] = ub;
            xbv[i][s] = vb;
            float2 pn = make_float2(0.f, 0.f);
            float4 qn = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q >= lo && q <= hi - 1) {
                const float ub_r = from_right(ub);
                const float2 vb_r = make_float2(from_right(vb.x), from_right(vb.y));
                if constexpr (CB)
                    dual_step<TGV>(p_in, q_in, t_q, flag(i), ub, vb, ub_r, vb_r, xbu[i][o], xbv[i][o], a0, a1,
                                   sgD[i] * a.sigma_n[i], sqn[i], pn, qn);
                else
                    dual_at<TGV>(p_in, q_in, t_q, flag(i), ub, vb, ub_r, vb_r, xbu[i][o], xbv[i][o], a0, a1,
                                 a.sigma_n[i], sqn[i], pn, qn);
                if (i == N - 1 && q >= y0 && q < y1) write_dual<TGV, S>(P, xs, q, pn, qn, nt);
            }
            yp[i][s] = pn;
            yq[i][s] = qn;
        }
    };
    for (int r = r_hi; r >= r_lo; r -= 2) {
        step(r, Par<0>());
        if (r - 1 >= r_lo) step(r - 1, Par<1>());
    }
}

// N iterations in one pass over memory.  Even segments march down, odd ones
// up, so that the halo rows two neighbouring segments share are read by both
// at the same time (both at the end of their marches, or both at the start)
// and the second read hits in L2.  Both marches call the same step functions
// on the same inputs, so each pixel's result does not depend on the
// direction (this file contracts multiply-adds only within one expression).
template <bool TGV, int S, int N, bool FIRST>
__global__ __launch_bounds__(kLanes * kWaves, N == 4 || (N == 3 && S == ST_F32) ? 3 : (S != ST_F32 ? 4 : 1)) void pdn_kernel(PdArgs a, int by,
                                                                                               int segs)
{
    constexpr int kColsN = kLanes - 2 * N;
    Task tk;
    if (!task_of(a, kColsN, by, segs, tk)) return;
    Planes P;
    if (!planes_of<S>(a, tk.pair, P)) return;
    const int tx = tk.tx;
    if (tx * kColsN >= P.W) return;

    const int lane = threadIdx.x & (kLanes - 1);
    const int x = tx * kColsN - N + lane;
    const bool owner = lane >= N && lane < N + kColsN && x < P.W;
    const int y0 = tk.y0;
    if (y0 >= P.H) return;
    const int y1 = min(y0 + by, P.H);
    // the four-iteration kernels' LDS ring of row constants (RowConsts): 2N
    // slots per wavefront, of which an upward march uses N
    using TRaw = typename TensorRaw<S>::type;
    constexpr int RW = N >= 4 ? kWaves : 1, RD = N >= 4 ? 2 * N : 1;
    __shared__ TRaw ringT[RW][RD][kLanes];
    __shared__ float ringR[RW][RD][kLanes];
    const int wv = N >= 4 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes) : 0;
    if ((y0 / by) & 1)
        march_up<TGV, S, N, FIRST>(a, P, x, owner, y0, y1, ringT[wv], ringR[wv]);
    else
        march_down<TGV, S, N, FIRST>(a, P, x, owner, y0, y1, ringT[wv], ringR[wv]);
}

// Wavefronts of a kernel that the current device holds at once (its
// occupancy times the compute units), cached per kernel and device.
template <typename K>
long long resident_waves(K kernel)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, long long> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), dev);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int blocks = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, kLanes * kWaves, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    const long long w = (long long)blocks * cus * kWaves;
    cache.emplace(key, w);
    return w;
}

// SIMDs of the current device (compute units x 4), cached per device.
long long device_simds()
{
    static std::mutex mu;
    static std::map<int, long long> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    const long long n = 4LL * cus;
    cache.emplace(dev, n);
    return n;
}

// Segment height, segment count and workgroups of a launch whose wavefronts
// own `cols` columns (blocks = 0: nothing to do).
struct March {
    int by, segs;
    long long blocks;
};

// The shortest march a launch may use.  Short marches cost halo rows; they
// pay where the launch cannot fill the SIMDs anyway and its time is one
// wavefront's chain of row steps: down to 1 row while the launch holds at
// most one wavefront per SIMD, to 2 rows while it holds at most two
// (measured on the 32x32 to 256x256 pyramid levels of 8 pairs: 16.4 -> 11.6,
// 16.6 -> 11.8 and 17.1 -> 16.0 us per three-iteration launch; shorter
// marches at 256x256 were slower; single-pair solves of 320x240 to 1024x768
// pairs one at a time: 73 -> 94 pairs/s).
int short_march_floor(const PdArgs& a, int cols)
{
    const long long H = a.lc.g.H[a.lc.gl];
    const long long strips = (long long)(a.lc.g.W[a.lc.gl] + cols - 1) / cols * a.lc.n;
    const long long simds = device_simds();
    if (strips * H <= simds) return 1;
    if (strips * ((H + 1) / 2) <= 2 * simds) return 2;
    return kBYs;
}

template <typename K>
March march_shape(const PdArgs& a, int cols, K kernel, int min_by = kBYs, int target_by = kBY)
{
    March m{0, 0, 0};
    const int H = a.lc.g.H[a.lc.gl];
    const long long strips = (long long)(a.lc.g.W[a.lc.gl] + cols - 1) / cols * a.lc.n;
    if (strips < 1 || H < 1) return m;
    const long long slots = resident_waves(kernel);
    const long long full = strips * ((H + target_by - 1) / target_by);
    long long segs;
    if (full >= kRoundsForShort * slots) {
        const long long rounds = (full + slots / 2) / slots;
        segs = rounds * slots / strips;
    } else {
        segs = slots / strips;
    }
    if (segs < 1) segs = 1;
    int by = int((H + segs - 1) / segs);
    if (by < min_by) by = min_by;
    m.by = by;
    m.segs = (H + by - 1) / by;
    m.blocks = (strips * m.segs + kWaves - 1) / kWaves;
    return m;
}

template <int MODE, bool TGV, int S>
void launch_mode(const PdArgs& a, hipStream_t s)
{
    const March m = march_shape(a, kCols, pd_kernel<MODE, TGV, S>, short_march_floor(a, kCols));
    if (m.blocks)
        hipLaunchKernelGGL((pd_kernel<MODE, TGV, S>), dim3(m.blocks), dim3(kLanes * kWaves), 0, s, a, m.by, m.segs);
}

// Bytes above which a multi-iteration pass's state cannot stay in the last
// level cache between passes (the 256 MB Infinity Cache of MI355X): its FP32
// passes then store it non-temporally, keeping L2 for the halo rows and
// columns that neighbouring marches re-read (measured on 8 pairs of
// 2048x2048: 700.0 -> 697.1 us per level-0 launch; with non-temporal stores
// everywhere, a cache-resident 1280x1024 pair went 31.2 -> 34.2 us and
// 16-bit storage on the 2048x2048 pairs 503 -> 540 us, so neither gets them).
constexpr long long kLastLevelCache = 256ll << 20;

template <bool TGV, int S, int N, bool FIRST>
void launch_fusedn(const PdArgs& a0, hipStream_t s)
{
    PdArgs a = a0;
    const long long state = (long long)a.lc.n * a.lc.g.W[a.lc.gl] * a.lc.g.H[a.lc.gl] * 93;
    a.nt_stores = S == ST_F32 && state > kLastLevelCache;
    const March m = march_shape(a, kLanes - 2 * N, pdn_kernel<TGV, S, N, FIRST>, short_march_floor(a, kLanes - 2 * N),
                                S == ST_F32 ? (N == 4 ? kBY4 : kBY) : kBY16);
    if (m.blocks)
        hipLaunchKernelGGL((pdn_kernel<TGV, S, N, FIRST>), dim3(m.blocks), dim3(kLanes * kWaves), 0, s, a, m.by, m.segs);
}

template <bool TGV, int S>
void launch_typed(const PdArgs& a, hipStream_t s)
{
    if (a.mode == PD_DUAL_FIRST) launch_mode<PD_DUAL_FIRST, TGV, S>(a, s);
    else if (a.mode == PD_FUSED) launch_mode<PD_FUSED, TGV, S>(a, s);
    else if (a.mode == PD_FUSED2) launch_fusedn<TGV, S, 2, false>(a, s);
    else if (a.mode == PD_FIRST2) launch_fusedn<TGV, S, 2, true>(a, s);
    else if (a.mode == PD_FUSED3) launch_fusedn<TGV, S, 3, false>(a, s);
    else if (a.mode == PD_FUSED4) launch_fusedn<TGV, S, 4, false>(a, s);
    else if (a.mode == PD_FIRST3) launch_fusedn<TGV, S, 3, true>(a, s);
    else if (a.mode == PD_FIRST4) launch_fusedn<TGV, S, 4, true>(a, s);
    else launch_mode<PD_PRIMAL_LAST, TGV, S>(a, s);
}

template <bool TGV, int S>
void prepare_typed()
{
    (void)resident_waves(pd_kernel<PD_DUAL_FIRST, TGV, S>);
    (void)resident_waves(pd_kernel<PD_FUSED, TGV, S>);
    (void)resident_waves(pd_kernel<PD_PRIMAL_LAST, TGV, S>);
    (void)resident_waves(pdn_kernel<TGV, S, 2, false>);
    (void)resident_waves(pdn_kernel<TGV, S, 2, true>);
    (void)resident_waves(pdn_kernel<TGV, S, 3, false>);
    (void)resident_waves(pdn_kernel<TGV, S, 4, false>);
    (void)resident_waves(pdn_kernel<TGV, S, 3, true>);
    (void)resident_waves(pdn_kernel<TGV, S, 4, true>);
}

}  // namespace

void prepare_pd()
{
    (void)device_simds();
    prepare_typed<true, ST_F32>();
    prepare_typed<true, ST_F16>();
    prepare_typed<true, ST_BF16>();
    prepare_typed<false, ST_F32>();
    prepare_typed<false, ST_F16>();
    prepare_typed<false, ST_BF16>();
}

void launch_pd(const PdArgs& a, hipStream_t s)
{
    if (a.tgv) {
        if (a.storage == ST_F16) launch_typed<true, ST_F16>(a, s);
        else if (a.storage == ST_BF16) launch_typed<true, ST_BF16>(a, s);
        else launch_typed<true, ST_F32>(a, s);
    } else {
        if (a.storage == ST_F16) launch_typed<false, ST_F16>(a, s);
        else if (a.storage == ST_BF16) launch_typed<false, ST_BF16>(a, s);
        else launch_typed<false, ST_F32>(a, s);
    }
}

}  // namespace vfs
