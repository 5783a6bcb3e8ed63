// Link metrics of RZF precoding from a solve with S = I_K (the paper's
// signal model and its RZF section, with Remark 1 for F = H^H V): row b of X
// is f_b, column b of the unnormalised precoding matrix F. Per problem:
//   E[u][b] = h_u^H f_b = sum over n in VR_u of H[u][n] X[b][n]
//   beta    = 1 / ||F||_F                      (power budget ||beta F||_F = 1)
//   R_u     = log2(1 + beta^2 |E_uu|^2 / (beta^2 sum_{b != u} |E_ub|^2 + xi))
// with xi = sigma^2 / rho, so the rate is the spectral efficiency of user u.
// E is a K x K product over the band: on the matrix cores from the residual
// tiles of the MFMA engine's plans, else tiled through LDS on the VALU;
// accumulated in the data type, the sums of the rates in double.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

template <typename R>
struct C {
    R x, y;
};

// E[u][b] for every problem, in 16 x 16 tiles: blockIdx.y is the problem,
// blockIdx.x the tile (16 users of VR-start order, 16 precoders). Chunks of
// 64 antennas of the users' band union and of the precoders' rows are staged
// in LDS (H zero outside each user's VR); thread (i, j) accumulates entry
// (user i, precoder j) over the chunk.
constexpr int kChunk = 64;

template <typename R>
__global__ void __launch_bounds__(256) k_link_effective(const VrkDesc *descs, const VrkLinkOut *outs, int tiles_1d)
{
    __shared__ C<R> hs[16][kChunk + 1], xs[16][kChunk + 1];
    __shared__ int band[2];
    const VrkDesc &d = descs[blockIdx.y];
    const int K = d.k, N = d.nt;
    const int tu = blockIdx.x / tiles_1d, tb = blockIdx.x % tiles_1d;
    if (tu * 16 >= K || tb * 16 >= K) return;   // the whole workgroup
    const int tid = threadIdx.x, i = tid >> 4, j = tid & 15;
    // this tile's users (original indices) and their band union
    if (tid == 0) {
        band[0] = N;
        band[1] = 0;
    }
    __syncthreads();
    const int su = tu * 16 + (tid & 15);
    if (tid < 16 && su < K) {
        const int u = d.perm[su];
        if (d.ve[u] > d.vs[u]) {
            atomicMin(&band[0], d.vs[u]);
            atomicMax(&band[1], d.ve[u]);
        }
    }
    __syncthreads();
    const int lo = band[0], hi = band[1];
    const C<R> *H = reinterpret_cast<const C<R> *>(d.H);
    const C<R> *X = reinterpret_cast<const C<R> *>(d.X);
    R re = 0, im = 0;
    for (int n0 = lo; n0 < hi; n0 += kChunk) {
        // 16 x 64 of H and of X: thread tid loads column tid % 64 of rows
        // tid / 64, tid / 64 + 4, ...
        const int c = tid & (kChunk - 1), n = n0 + c;
#pragma unroll
        for (int r = tid / kChunk; r < 16; r += 256 / kChunk) {
            C<R> hv = {0, 0}, xv = {0, 0};
            const int s2 = tu * 16 + r, b = tb * 16 + r;
            if (s2 < K && n < N) {
                const int u = d.perm[s2];
                if (n >= d.vs[u] && n < d.ve[u]) hv = H[(int64_t)u * d.ldh + n];
            }
            if (b < K && n < N) xv = X[(int64_t)b * d.ldx + n];
            hs[r][c] = hv;
            xs[r][c] = xv;
        }
        __syncthreads();
#pragma unroll 8
        for (int cc = 0; cc < kChunk; ++cc) {
            const C<R> a = hs[i][cc], x = xs[j][cc];
            re += a.x * x.x - a.y * x.y;
            im += a.x * x.y + a.y * x.x;
        }
        __syncthreads();
    }
    const int s2 = tu * 16 + i, b = tb * 16 + j;
    if (s2 < K && b < K) {
        const VrkLinkOut o = outs[blockIdx.y];
        reinterpret_cast<C<R> *>(o.E)[(int64_t)d.perm[s2] * o.lde + b] = C<R>{re, im};
    }
}

// beta and the rates, one workgroup per problem: ||X||_F^2 summed in a fixed
// order (thread t takes column t, t + 1024, ... of each row into one of
// eight partial sums by row, eight rows in flight, then a tree over the
// threads), then one user per thread.
template <typename R>
__global__ void __launch_bounds__(1024) k_link_rates(const VrkDesc *descs, const VrkLinkOut *outs)
{
    __shared__ double red[1024];
    const VrkDesc &d = descs[blockIdx.x];
    const VrkLinkOut o = outs[blockIdx.x];
    const int tid = threadIdx.x, K = d.k, N = d.nt;
    const C<R> *X = reinterpret_cast<const C<R> *>(d.X);
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int n = tid; n < N; n += 1024)
        for (int b0 = 0; b0 < K; b0 += 8) {
            C<R> v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                v[q] = C<R>{0, 0};
                if (b0 + q < K) v[q] = X[(int64_t)(b0 + q) * d.ldx + n];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += (double)v[q].x * v[q].x + (double)v[q].y * v[q].y;
        }
    red[tid] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    for (int m = 512; m > 0; m >>= 1) {
        if (tid < m) red[tid] += red[tid + m];
        __syncthreads();
    }
    const double fro2 = red[0];
    const double beta2 = fro2 > 0.0 ? 1.0 / fro2 : 0.0;
    if (tid == 0) o.beta[0] = fro2 > 0.0 ? 1.0 / sqrt(fro2) : 0.0;
    const C<R> *E = reinterpret_cast<const C<R> *>(o.E);
    for (int u = tid; u < K; u += 1024) {
        double sig = 0.0, intf = 0.0;
        for (int b = 0; b < K; ++b) {
            const C<R> v = E[(int64_t)u * o.lde + b];
            const double a2 = (double)v.x * v.x + (double)v.y * v.y;
            if (b == u) sig = a2;
            else intf += a2;
        }
        o.rate[u] = log2(1.0 + beta2 * sig / (beta2 * intf + d.xi));
    }
}

typedef float f4 __attribute__((ext_vector_type(4)));

// Sums of complex products with three real products each (Gauss):
// u += Ar Br, v += Ai Bi, w += (Ar + Ai)(Br + Bi); Re = u - v, Im = w - u - v.
struct C3 {
    f4 u, v, w;
};

__device__ __forceinline__ void c3mfma(C3 &acc, float2 a, float2 b)
{
    acc.u = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc.u, 0, 0, 0);
    acc.v = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc.v, 0, 0, 0);
    acc.w = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, acc.w, 0, 0, 0);
}

// E on the matrix cores (complex64, MFMA-engine plans): wave w of block x
// takes item 4 x + w = (user block ub, precoder block tb) of problem
// blockIdx.y. A = the residual tiles of ub (lane i + 16 kk of tile
// (ab, m) holds H[16 ub + i][16 ab + 4 kk + m], zero off the VRs), B = rows
// 16 tb + j of X at antennas 16 ab + 4 kk + m; four antenna blocks' loads
// in flight at a time.
__global__ void __launch_bounds__(256) k_link_effective_mfma(const VrkDesc *descs, const VrkLinkOut *outs)
{
    const VrkDesc &d = descs[blockIdx.y];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int K = d.k, nub = d.nub, ntb = (K + 15) / 16;
    const int item = blockIdx.x * 4 + w;
    if (item >= nub * ntb) return;
    const int ub = __builtin_amdgcn_readfirstlane(item / ntb), tb = __builtin_amdgcn_readfirstlane(item % ntb);
    const int lo = __builtin_amdgcn_readfirstlane(d.rab_lo[ub]), hi = __builtin_amdgcn_readfirstlane(d.rab_hi[ub]);
    const float2 *ha = reinterpret_cast<const float2 *>(d.HA) + d.ha_off[ub] * 64 + lane;
    const int b = tb * 16 + j, N = d.nt;
    const float2 *xrow = reinterpret_cast<const float2 *>(d.X) + (int64_t)(b < K ? b : 0) * d.ldx;
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc = {z, z, z};
    for (int ab0 = lo; ab0 < hi; ab0 += 4) {
        float2 h[4][4], x[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ab = ab0 + t;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int n = 16 * ab + 4 * g + m;
                h[t][m] = x[t][m] = float2{0.f, 0.f};
                if (ab < hi) {
                    h[t][m] = ha[(int64_t)(4 * (ab - lo) + m) * 64];
                    if (b < K && n < N) x[t][m] = xrow[n];
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (ab0 + t < hi)
#pragma unroll
                for (int m = 0; m < 4; ++m) c3mfma(acc, h[t][m], x[t][m]);
    }
    // D layout: lane (j, g) register r holds user 16 ub + 4 g + r, precoder 16 tb + j
    const VrkLinkOut o = outs[blockIdx.y];
    const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int su = ub * 16 + 4 * g + r;
        if (su < K && b < K)
            reinterpret_cast<float2 *>(o.E)[(int64_t)d.perm[su] * o.lde + b] = float2{re[r], im[r]};
    }
}

}  // namespace

hipError_t vrk_launch_link(const VrkDesc *desc, const VrkLinkOut *outs, int32_t nprob, int32_t max_k, int32_t dtype,
                           int32_t mfma, hipStream_t s)
{
    if (nprob <= 0 || max_k <= 0) return hipSuccess;
    if (mfma && dtype == 0) {
        const int nt1 = (max_k + 15) / 16;
        hipLaunchKernelGGL(k_link_effective_mfma, dim3((unsigned)((nt1 * nt1 + 3) / 4), (unsigned)nprob), dim3(256), 0,
                           s, desc, outs);
        hipLaunchKernelGGL(k_link_rates<float>, dim3(nprob), dim3(1024), 0, s, desc, outs);
        return hipGetLastError();
    }
    const int t1 = (max_k + 15) / 16;
    const dim3 ge((unsigned)(t1 * t1), (unsigned)nprob);
    if (dtype == 1) {
        hipLaunchKernelGGL(k_link_effective<double>, ge, dim3(256), 0, s, desc, outs, t1);
        hipLaunchKernelGGL(k_link_rates<double>, dim3(nprob), dim3(1024), 0, s, desc, outs);
    } else {
        hipLaunchKernelGGL(k_link_effective<float>, ge, dim3(256), 0, s, desc, outs, t1);
        hipLaunchKernelGGL(k_link_rates<float>, dim3(nprob), dim3(1024), 0, s, desc, outs);
    }
    return hipGetLastError();
}
