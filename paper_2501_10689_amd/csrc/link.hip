// Link metrics of RZF precoding from a solve with S = I_K (the paper's
// signal model and its RZF section, with Remark 1 for F = H^H V): row b of X
// is f_b, column b of the unnormalised precoding matrix F. Per problem:
//   E[u][b] = h_u^H f_b = sum over n in VR_u of H[u][n] X[b][n]
//   beta    = 1 / ||F||_F                      (power budget ||beta F||_F = 1)
//   R_u     = log2(1 + beta^2 |E_uu|^2 / (beta^2 sum_{b != u} |E_ub|^2 + sigma^2 / rho))
// with sigma^2 / rho given per problem (the output table's noise), so the
// rate is the spectral efficiency of user u.
// On MFMA-engine plans X = H^H V exactly (the solve forms x from its dual
// iterate q = v), so E = H H^H V^T = (M - xi I) V^T: a K x K x K product
// with the Gram tiles instead of a band product over the antennas. Vector
// engine plans take the band product, tiled through LDS. ||X||_F^2 is summed
// from X itself in double, in a fixed order, over VRK_LINK_GROUPS
// workgroups per problem.
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

// Partial sums of ||X||_F^2: workgroup (p, y) adds |X[b][n]|^2 in double
// over the rows b = y, y + VRK_LINK_GROUPS, ... of problem p (thread t the
// columns t + 256 q + 1024 i into accumulator q), then a tree
// over the threads; the partial goes to part[p * VRK_LINK_GROUPS + y].
template <typename R>
__global__ void __launch_bounds__(256) k_link_fro(const VrkDesc *descs, double *part)
{
    __shared__ double red[256];
    const VrkDesc &d = descs[blockIdx.x];
    const int tid = threadIdx.x, K = d.k, N = d.nt;
    const C<R> *X = reinterpret_cast<const C<R> *>(d.X);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = blockIdx.y; b < K; b += VRK_LINK_GROUPS) {
        const C<R> *row = X + (int64_t)b * d.ldx;
        for (int n0 = tid; n0 < N; n0 += 1024) {
            C<R> v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = n0 + 256 * q < N ? row[n0 + 256 * q] : C<R>{0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += (double)v[q].x * v[q].x + (double)v[q].y * v[q].y;
        }
    }
    red[tid] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if (tid < m) red[tid] += red[tid + m];
        __syncthreads();
    }
    if (tid == 0) part[(int64_t)blockIdx.x * VRK_LINK_GROUPS + blockIdx.y] = red[0];
}

// beta and the rates, one workgroup per problem: ||X||_F^2 = the partials
// added in group order, then one user per thread.
template <typename R>
__global__ void __launch_bounds__(256) k_link_rates(const VrkDesc *descs, const VrkLinkOut *outs, const double *part)
{
    const VrkDesc &d = descs[blockIdx.x];
    const VrkLinkOut o = outs[blockIdx.x];
    const int K = d.k;
    double fro2 = 0.0;
    for (int y = 0; y < VRK_LINK_GROUPS; ++y) fro2 += part[(int64_t)blockIdx.x * VRK_LINK_GROUPS + y];
    const double beta2 = fro2 > 0.0 ? 1.0 / fro2 : 0.0;
    if (threadIdx.x == 0) o.beta[0] = fro2 > 0.0 ? 1.0 / sqrt(fro2) : 0.0;
    const C<R> *E = reinterpret_cast<const C<R> *>(o.E);
    for (int u = threadIdx.x; u < K; u += 256) {
        double sig = 0.0, intf = 0.0;
        for (int b = 0; b < K; ++b) {
            const C<R> v = E[(int64_t)u * o.lde + b];
            const double a2 = (double)v.x * v.x + (double)v.y * v.y;
            if (b == u) sig = a2;
            else intf += a2;
        }
        o.rate[u] = log2(1.0 + beta2 * sig / (beta2 * intf + o.noise));
    }
}

// E on the matrix cores (complex64, MFMA-engine plans): workgroup x of
// problem blockIdx.y takes precoder block tb = x % ntb and user blocks
// mb = 4 (x / ntb) + w (one per wave). The workgroup stages rows 16 tb .. +15
// of V in LDS with the users in VR-start order, then each wave multiplies
// the Gram tiles of its row block (A: lane i + 16 kk of tile e holds
// M[16 mb + i][4 c + kk], only the chunks c of the block pattern, so M is
// zero elsewhere) by B[kk][j] = V[16 tb + j][perm[4 c + kk]] and subtracts
// xi V. Rows of users without any visible antenna are written as zero (their
// row of M is xi e_u).
constexpr int kLinkUsers = 16 * 16;   // users per problem on the MFMA engine (16 waves x 16)

__global__ void __launch_bounds__(256) k_link_effective_gram(const VrkDesc *descs, const VrkLinkOut *outs)
{
    __shared__ float2 vsrt[16][kLinkUsers + 1];
    const VrkDesc &d = descs[blockIdx.y];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int K = d.k, nub = d.nub, ntb = (K + 15) / 16, kpad = nub * 16;
    if ((int)blockIdx.x >= ntb * ((nub + 3) / 4)) return;   // the whole workgroup
    const int tb = blockIdx.x % ntb, mb = (blockIdx.x / ntb) * 4 + w;
    const float2 *V = reinterpret_cast<const float2 *>(d.V);
    for (int t = threadIdx.x; t < 16 * kpad; t += 256) {
        const int jj = t / kpad, ks = t % kpad, bb = tb * 16 + jj;
        vsrt[jj][ks] = (bb < K && ks < K) ? V[(int64_t)bb * d.ldv + d.perm[ks]] : float2{0.f, 0.f};
    }
    __syncthreads();
    if (mb >= nub) return;
    const int e0 = d.gm_off[mb], e1 = d.gm_off[mb + 1];
    const float2 *gm = reinterpret_cast<const float2 *>(d.GM) + lane;
    const int b = tb * 16 + j;
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc = {z, z, z};
    for (int e = e0; e < e1; e += 4) {   // the lists are padded to groups of four
        float2 a[4], v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = d.gm_c[e + t];   // -1: padding chunk, zero tile
            a[t] = gm[(int64_t)(e + t) * 64];
            v[t] = c >= 0 ? vsrt[j][4 * c + g] : float2{0.f, 0.f};
        }
        __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
        for (int t = 0; t < 4; ++t) c3mfma(acc, a[t], v[t]);
    }
    // D layout: lane (j, g) register r holds user 16 mb + 4 g + r, precoder 16 tb + j
    const VrkLinkOut o = outs[blockIdx.y];
    const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
    const float xi = (float)d.xi;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int su = mb * 16 + 4 * g + r;
        if (su < K && b < K) {
            const int u = d.perm[su];
            float2 ev = {0.f, 0.f};
            if (d.ve[u] > d.vs[u]) {
                const float2 q = vsrt[j][su];
                ev = float2{re[r] - xi * q.x, im[r] - xi * q.y};
            }
            reinterpret_cast<float2 *>(o.E)[(int64_t)u * o.lde + b] = ev;
        }
    }
}

}  // namespace

hipError_t vrk_launch_link(const VrkDesc *desc, const VrkLinkOut *outs, int32_t nprob, int32_t max_k, int32_t dtype,
                           int32_t mfma, double *part, hipStream_t s)
{
    if (nprob <= 0 || max_k <= 0) return hipSuccess;
    const dim3 gf((unsigned)nprob, VRK_LINK_GROUPS);
    if (mfma && dtype == 0) {
        const int nt1 = (max_k + 15) / 16;
        hipLaunchKernelGGL(k_link_effective_gram, dim3((unsigned)(nt1 * ((nt1 + 3) / 4)), (unsigned)nprob), dim3(256),
                           0, s, desc, outs);
        hipLaunchKernelGGL(k_link_fro<float>, gf, dim3(256), 0, s, desc, part);
        hipLaunchKernelGGL(k_link_rates<float>, dim3(nprob), dim3(256), 0, s, desc, outs, part);
        return hipGetLastError();
    }
    const int t1 = (max_k + 15) / 16;
    const dim3 ge((unsigned)(t1 * t1), (unsigned)nprob);
    if (dtype == 1) {
        hipLaunchKernelGGL(k_link_effective<double>, ge, dim3(256), 0, s, desc, outs, t1);
        hipLaunchKernelGGL(k_link_fro<double>, gf, dim3(256), 0, s, desc, part);
        hipLaunchKernelGGL(k_link_rates<double>, dim3(nprob), dim3(256), 0, s, desc, outs, part);
    } else {
        hipLaunchKernelGGL(k_link_effective<float>, ge, dim3(256), 0, s, desc, outs, t1);
        hipLaunchKernelGGL(k_link_fro<float>, gf, dim3(256), 0, s, desc, part);
        hipLaunchKernelGGL(k_link_rates<float>, dim3(nprob), dim3(256), 0, s, desc, outs, part);
    }
    return hipGetLastError();
}
