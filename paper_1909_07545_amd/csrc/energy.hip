// Linearised energy of Eq. (10) at one level and one warp,
//   E = sum over the mask of  lambda |rho_c + u I_u|  +  alpha1 |T grad u - v|_2
//                            + alpha0 |grad v|_F      (TGV; v = 0 and no last term for TV),
// with the masked forward differences of the primal-dual iteration, and the
// difference statistics of two planes.  Per-pixel terms are FP32 (the
// solver's precision), accumulated in FP64 by a fixed-order two-pass
// reduction (wavefront lanes by xor-shuffles, the 4 wavefronts of a
// workgroup in order, then one workgroup over the per-workgroup partials), so
// the result does not depend on scheduling.
#include "vfs_internal.h"

namespace vfs {

namespace {

constexpr int kRows = 4;    // rows per workgroup (one 64-lane wavefront each)

__device__ inline double wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ inline double wave_max(double x)
{
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// Workgroup of 4 x 64: partial[block] = sum of the lanes' values.
__device__ inline void block_store(double x, double* partial, size_t slot)
{
    __shared__ double part[kRows];
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) partial[slot] = ((part[0] + part[1]) + part[2]) + part[3];
    __syncthreads();    // part[] is reused by the next call
}

template <int S>
__global__ void energy_kernel(Launch lc, float lambda, float a0, float a1, int tgv, double* partial)
{
    const int z = blockIdx.z;
    const size_t slot = ((size_t)z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    Pick pk;
    double e = 0.0;
    if (pick(lc, z, pk)) {
        const Slot& sl = lc.slots[pk.slot];
        const int l = pk.l, W = lc.g.W[l], H = lc.g.H[l], pitch = lc.g.pitch[l];
        const int j = blockIdx.x * 64 + (threadIdx.x & 63);
        const int i = blockIdx.y * kRows + (threadIdx.x >> 6);
        if (j < W && i < H) {
            const size_t o = (size_t)i * pitch + j;
            const unsigned f = sl.flags[l][o];
            if (f & F_MASK) {
                const int pu = (lc.iu ^ int(pk.flip)) & 1;
                const float* u = sl.u[pu] + lc.g.off[l];
                const float mx = (f & F_MX) ? 1.f : 0.f, my = (f & F_MY) ? 1.f : 0.f;
                const float uc = u[o];
                const float gx = (f & F_MX) ? u[o + 1] - uc : 0.f;
                const float gy = (f & F_MY) ? u[o + pitch] - uc : 0.f;
                const float4 t = ld4<S>(sl.tpack, o);
                float2 vc = make_float2(0.f, 0.f);
                const float2* v = nullptr;
                if (tgv) {
                    v = sl.v[pu] + lc.g.off[l];
                    vc = v[o];
                }
                const float b1 = t.x * gx + t.y * gy - vc.x, b2 = t.y * gx + t.z * gy - vc.y;
                float ep = lambda * fabsf(sl.rho[o] + uc * t.w) + a1 * sqrtf(b1 * b1 + b2 * b2);
                if (tgv) {
                    const float2 vr = (f & F_MX) ? v[o + 1] : vc, vd = (f & F_MY) ? v[o + pitch] : vc;
                    const float d11 = mx * (vr.x - vc.x), d12 = my * (vd.x - vc.x);
                    const float d21 = mx * (vr.y - vc.y), d22 = my * (vd.y - vc.y);
                    ep += a0 * sqrtf(d11 * d11 + d12 * d12 + d21 * d21 + d22 * d22);
                }
                e = double(ep);
            }
        }
    }
    block_store(e, partial, slot);
}

// |a - b| over the pixels with mask bit set in `mask` (or all if NULL):
// partial sums of |a - b| and of the count, and per-workgroup maxima.
__global__ void diff_kernel(int W, int H, int pitch, const float* a, const float* b, const uint8_t* mask,
                            double* psum, double* pmax, double* pcnt)
{
    const size_t slot = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * kRows + (threadIdx.x >> 6);
    double d = 0.0, c = 0.0;
    if (j < W && i < H) {
        const size_t o = (size_t)i * pitch + j;
        if (!mask || (mask[o] & F_MASK)) {
            d = fabs(double(a[o]) - double(b[o]));
            c = 1.0;
        }
    }
    __shared__ double mx[kRows];
    const double m = wave_max(d);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) mx[wave] = m;
    block_store(d, psum, slot);
    block_store(c, pcnt, slot);
    if (threadIdx.x == 0) pmax[slot] = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
}

// out[k] = sum (or max) of in[k * n .. k * n + n - 1], for k < m; one workgroup per k.
__global__ void finish_kernel(const double* in, long long n, int use_max, double* out)
{
    __shared__ double part[256];
    const double* p = in + (size_t)blockIdx.x * n;
    double x = 0.0;
    for (long long k = threadIdx.x; k < n; k += 256) x = use_max ? fmax(x, p[k]) : x + p[k];
    part[threadIdx.x] = x;
    __syncthreads();
    for (unsigned s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            part[threadIdx.x] = use_max ? fmax(part[threadIdx.x], part[threadIdx.x + s])
                                        : part[threadIdx.x] + part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

}  // namespace

size_t energy_partials(const Launch& lc)
{
    const int W = lc.g.W[lc.gl], H = lc.g.H[lc.gl];
    return size_t((W + 63) / 64) * size_t((H + kRows - 1) / kRows) * size_t(lc.n);
}

void launch_energy(const Launch& lc, const EnergyConsts& k, double* partial, double* out, hipStream_t s)
{
    const int W = lc.g.W[lc.gl], H = lc.g.H[lc.gl];
    const dim3 grid((W + 63) / 64, (H + kRows - 1) / kRows, lc.n);
    if (k.storage == ST_F16)
        hipLaunchKernelGGL(energy_kernel<ST_F16>, grid, dim3(64 * kRows), 0, s, lc, k.lambda, k.alpha0, k.alpha1,
                           k.tgv, partial);
    else if (k.storage == ST_BF16)
        hipLaunchKernelGGL(energy_kernel<ST_BF16>, grid, dim3(64 * kRows), 0, s, lc, k.lambda, k.alpha0, k.alpha1,
                           k.tgv, partial);
    else
        hipLaunchKernelGGL(energy_kernel<ST_F32>, grid, dim3(64 * kRows), 0, s, lc, k.lambda, k.alpha0, k.alpha1,
                           k.tgv, partial);
    // one sum per pair
    const long long per = (long long)grid.x * grid.y;
    hipLaunchKernelGGL(finish_kernel, dim3(lc.n), dim3(256), 0, s, partial, per, 0, out);
}

size_t diff_partials(int W, int H) { return size_t((W + 63) / 64) * size_t((H + kRows - 1) / kRows); }

void launch_diff_stats(int W, int H, int pitch, const float* a, const float* b, const uint8_t* mask,
                       double* partial, double* out3, hipStream_t s)
{
    const dim3 grid((W + 63) / 64, (H + kRows - 1) / kRows);
    const size_t n = diff_partials(W, H);
    hipLaunchKernelGGL(diff_kernel, grid, dim3(64 * kRows), 0, s, W, H, pitch, a, b, mask, partial,
                       partial + n, partial + 2 * n);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, partial, (long long)n, 0, out3);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, partial + n, (long long)n, 1, out3 + 1);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, partial + 2 * n, (long long)n, 0, out3 + 2);
}

}  // namespace vfs
