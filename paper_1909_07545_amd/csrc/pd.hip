// Primal-dual iteration of the tensor-weighted TGV-L1 energy (Eq. (10)) by
// the Chambolle-Pock scheme of Eq. (11), with the diagonal preconditioning of
// Sec. III-D and the resolvent of Eq. (13).
//
// Iterates: the same sequence as the textbook order
//     y^{k+1} = P(y^k + sigma K xbar^k),  x^{k+1} = prox(x^k - tau K^T y^{k+1}),
//     xbar^{k+1} = x^{k+1} + theta (x^{k+1} - x^k),
// with x = (u, v), y = (p, q), but the state in memory is stored one half
// step apart, (x^{k-1}, y^k).  One launch (PD_FUSED) computes x^k on the
// tile plus a one-pixel halo, forms xbar^k in registers and finishes with
// y^{k+1}; xbar never touches memory.  A warp's K iterations are one
// PD_DUAL_FIRST launch (y^1 from x^0 = xbar^0), K-1 PD_FUSED launches and one
// PD_PRIMAL_LAST launch (x^K).  Every launch reads one copy of the state and
// writes the other.
//
// Work decomposition: one 64-lane wavefront owns 62 columns (lanes 1..62;
// lanes 0 and 63 are the x-halo) and marches down BY rows plus a one-row
// halo above and below, keeping the previous row's values in registers and
// exchanging x-neighbours by lane shuffles.  A workgroup holds 4 wavefronts
// stacked vertically.  Workgroups are renumbered so that the blocks the
// dispatcher places on one XCD cover a contiguous band of tiles (their halo
// re-reads then hit that XCD's L2).
#include "vfs_internal.h"

namespace vfs {

namespace {

constexpr int kLanes = 64;
constexpr int kCols = kLanes - 2;   // interior columns per wavefront
constexpr int kWaves = 4;           // wavefronts per workgroup
constexpr int kBY = 16;             // rows per wavefront
constexpr int kXcds = 8;

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float from_left(float x) { return __shfl_up(x, 1, kLanes); }
__device__ inline float from_right(float x) { return __shfl_down(x, 1, kLanes); }

struct Row {
    float u;
    float2 v, p;
    float4 q, t;   // t = (t11, t12, t22, I_u)
    float rho;
    unsigned f;
};

template <bool TGV, bool PRIMAL>
__device__ inline Row load_row(const PdArgs& a, long long base, int x, int r, bool in_x)
{
    Row w;
    w.u = 0.f; w.rho = 0.f; w.f = 0u;
    w.v = make_float2(0.f, 0.f);
    w.p = make_float2(0.f, 0.f);
    w.q = make_float4(0.f, 0.f, 0.f, 0.f);
    w.t = make_float4(1.f, 0.f, 1.f, 0.f);
    if (in_x && r >= 0 && r < a.H) {
        const size_t o = base + (size_t)r * a.pitch + x;
        w.u = a.u_in[o];
        w.p = a.p_in[o];
        w.t = a.tpack[o];
        w.f = a.flags[(size_t)r * a.pitch + x];
        if (PRIMAL) w.rho = a.rho[o];
        if (TGV) {
            w.v = a.v_in[o];
            w.q = a.q_in[o];
        }
    }
    return w;
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
    return uhat - rb / Iu;
}

template <int MODE, bool TGV>
__global__ __launch_bounds__(kLanes * kWaves) void pd_kernel(PdArgs a)
{
    constexpr bool PRIMAL = MODE != PD_DUAL_FIRST;
    constexpr bool DUAL = MODE != PD_PRIMAL_LAST;

    // XCD-aware renumbering of the workgroup
    const int nb = gridDim.x, bid = blockIdx.x;
    const int xcd = bid % kXcds, k = bid / kXcds, qn = nb / kXcds, rn = nb % kXcds;
    const int logical = xcd < rn ? xcd * (qn + 1) + k : rn * (qn + 1) + (xcd - rn) * qn + k;

    const int tiles_x = (a.W + kCols - 1) / kCols;
    const int tiles_y = (a.H + kBY * kWaves - 1) / (kBY * kWaves);
    const int tx = logical % tiles_x;
    const int ty = (logical / tiles_x) % tiles_y;
    const int pair = logical / (tiles_x * tiles_y);
    if (pair >= a.n) return;

    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = threadIdx.x / kLanes;
    const int x = tx * kCols - 1 + lane;
    const bool in_x = x >= 0 && x < a.W;
    const bool owner = lane >= 1 && lane <= kCols && in_x;
    const int y0 = (ty * kWaves + wave) * kBY;
    if (y0 >= a.H) return;
    const int y1 = min(y0 + kBY, a.H);          // owned rows [y0, y1)
    const long long base = (long long)pair * a.stride;

    const float a0 = a.alpha0, a1 = a.alpha1;
    const float ts = a.tau_scale, ss = a.sigma_scale, th = a.theta;
    const float sq = ss / (2.f * a0);           // sigma_q, scaled

    // values of the previous row
    float2 p_prev = make_float2(0.f, 0.f);
    float4 q_prev = make_float4(0.f, 0.f, 0.f, 0.f), t_prev = make_float4(1.f, 0.f, 1.f, 0.f);
    unsigned f_prev = 0u;
    float ub_prev = 0.f;
    float2 vb_prev = make_float2(0.f, 0.f);
    float b_prev = 0.f, cy_prev = 0.f, my_prev = 0.f, myq2_prev = 0.f, myq4_prev = 0.f;

    if (PRIMAL) {
        // row y0 - 1: only what the primal step of row y0 reads from above
        const Row w = load_row<TGV, false>(a, base, x, y0 - 1, in_x);
        const float my = (w.f & F_MY) ? 1.f : 0.f;
        b_prev = my * (w.t.y * w.p.x + w.t.z * w.p.y);
        cy_prev = my * (fabsf(w.t.y) + fabsf(w.t.z));
        my_prev = my;
        myq2_prev = my * w.q.y;
        myq4_prev = my * w.q.w;
    }

    const int r_end = DUAL ? y1 : y1 - 1;       // last row visited (row y1 is the look-ahead)
    for (int r = y0; r <= r_end; ++r) {
        const Row c = load_row<TGV, PRIMAL>(a, base, x, r, in_x);
        const float mx = (c.f & F_MX) ? 1.f : 0.f;
        const float my = (c.f & F_MY) ? 1.f : 0.f;
        const bool msk = (c.f & F_MASK) != 0u;

        // ---- primal step at row r: x^k from x^{k-1} and y^k
        float un = c.u;
        float2 vn = c.v;
        const float b = my * (c.t.y * c.p.x + c.t.z * c.p.y);
        const float cy = my * (fabsf(c.t.y) + fabsf(c.t.z));
        const float myq2 = my * c.q.y, myq4 = my * c.q.w;
        if (PRIMAL) {
            const float ax = mx * (c.t.x * c.p.x + c.t.y * c.p.y);
            const float cx = mx * (fabsf(c.t.x) + fabsf(c.t.y));
            const float ax_l = from_left(ax);
            const float cx_l = from_left(cx);
            const float divtp = ax - ax_l + b - b_prev;
            const float cu = fabsf(c.t.x * mx + c.t.y * my) + fabsf(c.t.y * mx + c.t.z * my) + cx_l + cy_prev;
            const float tau_u = (cu > 0.f ? frcp(a1 * cu) : frcp(a1)) * ts;
            const float uh = c.u + tau_u * a1 * divtp;
            const float ur = resolvent(uh, c.rho, c.t.w, tau_u, a.lambda);
            float2 vr = c.v;
            if (TGV) {
                const float mxq1 = mx * c.q.x, mxq3 = mx * c.q.z;
                const float mxq1_l = from_left(mxq1), mxq3_l = from_left(mxq3), mx_l = from_left(mx);
                const float d1 = mxq1 - mxq1_l + myq2 - myq2_prev;
                const float d2 = mxq3 - mxq3_l + myq4 - myq4_prev;
                const float tau_v = frcp(a1 + a0 * (mx + my + mx_l + my_prev)) * ts;
                vr.x = c.v.x + tau_v * (a1 * c.p.x + a0 * d1);
                vr.y = c.v.y + tau_v * (a1 * c.p.y + a0 * d2);
            }
            if (msk) { un = ur; vn = vr; }
            if (owner && r < y1) {
                const size_t o = base + (size_t)r * a.pitch + x;
                a.u_out[o] = un;
                if (TGV) a.v_out[o] = vn;
            }
        }
        // over-relaxation (xbar stays in registers)
        const float ub = un + th * (un - c.u);
        const float2 vb = make_float2(vn.x + th * (vn.x - c.v.x), vn.y + th * (vn.y - c.v.y));

        // ---- dual step at row r - 1: y^{k+1} from y^k and xbar^k
        if (DUAL) {
            const float ub_r = from_right(ub_prev);
            const float vb1_r = from_right(vb_prev.x), vb2_r = from_right(vb_prev.y);
            if (r > y0 && owner && (f_prev & F_MASK)) {
                const float pmx = (f_prev & F_MX) ? 1.f : 0.f;
                const float pmy = (f_prev & F_MY) ? 1.f : 0.f;
                const float4 t = t_prev;
                const float gx = pmx * (ub_r - ub_prev), gy = pmy * (ub - ub_prev);
                const float s1 = a1 * (fabsf(t.x * pmx + t.y * pmy) + fabsf(t.x) * pmx + fabsf(t.y) * pmy) +
                                 (TGV ? a1 : 0.f);
                const float s2 = a1 * (fabsf(t.y * pmx + t.z * pmy) + fabsf(t.y) * pmx + fabsf(t.z) * pmy) +
                                 (TGV ? a1 : 0.f);
                const float smax = fmaxf(s1, s2);
                const float sig = (smax > 0.f ? frcp(smax) : frcp(a1)) * ss;
                float p1 = p_prev.x + sig * a1 * (t.x * gx + t.y * gy - (TGV ? vb_prev.x : 0.f));
                float p2 = p_prev.y + sig * a1 * (t.y * gx + t.z * gy - (TGV ? vb_prev.y : 0.f));
                const float n2 = p1 * p1 + p2 * p2;
                if (n2 > 1.f) {
                    const float inv = __builtin_amdgcn_rsqf(n2);
                    p1 *= inv;
                    p2 *= inv;
                }
                const size_t o = base + (size_t)(r - 1) * a.pitch + x;
                a.p_out[o] = make_float2(p1, p2);
                if (TGV) {
                    float q1 = q_prev.x + sq * a0 * pmx * (vb1_r - vb_prev.x);
                    float q2 = q_prev.y + sq * a0 * pmy * (vb.x - vb_prev.x);
                    float q3 = q_prev.z + sq * a0 * pmx * (vb2_r - vb_prev.y);
                    float q4 = q_prev.w + sq * a0 * pmy * (vb.y - vb_prev.y);
                    const float m2 = q1 * q1 + q2 * q2 + q3 * q3 + q4 * q4;
                    if (m2 > 1.f) {
                        const float inv = __builtin_amdgcn_rsqf(m2);
                        q1 *= inv; q2 *= inv; q3 *= inv; q4 *= inv;
                    }
                    a.q_out[o] = make_float4(q1, q2, q3, q4);
                }
            } else if (r > y0 && owner) {
                // outside the mask the duals stay as they are (zero)
                const size_t o = base + (size_t)(r - 1) * a.pitch + x;
                a.p_out[o] = p_prev;
                if (TGV) a.q_out[o] = q_prev;
            }
        }

        // ---- slide the window
        p_prev = c.p;
        q_prev = c.q;
        t_prev = c.t;
        f_prev = c.f;
        ub_prev = ub;
        vb_prev = vb;
        b_prev = b;
        cy_prev = cy;
        my_prev = my;
        myq2_prev = myq2;
        myq4_prev = myq4;
    }
}

template <int MODE, bool TGV>
void launch_mode(const PdArgs& a, hipStream_t s)
{
    const int tiles_x = (a.W + kCols - 1) / kCols;
    const int tiles_y = (a.H + kBY * kWaves - 1) / (kBY * kWaves);
    const int nb = tiles_x * tiles_y * a.n;
    hipLaunchKernelGGL((pd_kernel<MODE, TGV>), dim3(nb), dim3(kLanes * kWaves), 0, s, a);
}

}  // namespace

void launch_pd(const PdArgs& a, hipStream_t s)
{
    if (a.tgv) {
        if (a.mode == PD_DUAL_FIRST) launch_mode<PD_DUAL_FIRST, true>(a, s);
        else if (a.mode == PD_FUSED) launch_mode<PD_FUSED, true>(a, s);
        else launch_mode<PD_PRIMAL_LAST, true>(a, s);
    } else {
        if (a.mode == PD_DUAL_FIRST) launch_mode<PD_DUAL_FIRST, false>(a, s);
        else if (a.mode == PD_FUSED) launch_mode<PD_FUSED, false>(a, s);
        else launch_mode<PD_PRIMAL_LAST, false>(a, s);
    }
}

}  // namespace vfs
