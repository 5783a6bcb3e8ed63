// Adjoint (implicit differentiation) gradient products of the MFMA engine,
// complex64.
//
// For x = H^H (H H^H + xi I)^-1 s and an incoming gradient g = 2 dL/d conj(x):
//   GH = sum_b v_b (g_b - xh_b)^H - mu_b x_b^H  on the VR band entries
//   gxi = -Re sum_b mu_b^H v_b
// with mu = (H H^H + xi I)^-1 H g and xh = H^H mu from the adjoint solve
// (whose right-hand side b = H g the solve kernel forms itself). The
// products run on v_mfma_f32_16x16x4f32 over the band tiles of the plan.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Sums of complex products with three real products each (Gauss):
// u += Ar Br, v += Ai Bi, w += (Ar + Ai)(Br + Bi); Re = u - v, Im = w - u - v.
struct C3 {
    f4 u, v, w;
};

__device__ __forceinline__ void c3mfma(C3 &acc, float2 a, float2 b)
{
    acc.u = mfma(a.x, b.x, acc.u);
    acc.v = mfma(a.y, b.y, acc.v);
    acc.w = mfma(a.x + a.y, b.x + b.y, acc.w);
}

using CDesc = const VRK_CONST VrkDesc;
template <typename T>
using gp = VRK_GLOBAL T *;

// GH on the band tiles (ub, ab) of the user blocks ub = 4 ubg .. 4 ubg + 3
// that meet antenna block ab: D[user i][antenna j] = sum_b A[i][b] B[b][j]
// with A = V^T, B = conj(GX - Xadj) plus A = -M^T, B = conj(X). A wave loads
// the antenna operands of 4 RHS once for all blocks of the group; v and mu
// come from the VR-start-order copies (16 users = 128 contiguous bytes).
// The RHS range is split over the waves and reduced through LDS.
constexpr int kGW = 4;
constexpr int kUG = VRK_GRAD_UG;

// Returns the lane's share of sum conj(mu) v over the users of the blocks
// whose first antenna block is ab (each (user, RHS) pair is counted in
// exactly one tile; users with an empty VR have mu = 0).
__device__ __forceinline__ float grads_group(CDesc &d, int ubg, int ab, int bs0, int be0,
                                             float2 (*part)[kUG][256], gp<float2> out)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 15, kk = lane >> 4;
    const gp<const float2> VS = gmem(static_cast<const float2 *>(d.Vsrt));
    const gp<const float2> MS = gmem(static_cast<const float2 *>(d.Msrt));
    const gp<const float2> GX = gmem(static_cast<const float2 *>(d.GX));
    const gp<const float2> XA = gmem(static_cast<const float2 *>(d.Xadj));
    const gp<const float2> X = gmem(static_cast<const float2 *>(d.X));
    const int64_t ldgx = d.ldgx, ldx = d.ldx, ldxa = d.nt;
    const int nub = d.nub, kpad = nub * VRK_UB;
    const int ub0 = ubg * kUG;
    // blocks of the group that meet ab (wave-uniform)
    bool live[kUG], first[kUG];
#pragma unroll
    for (int u = 0; u < kUG; ++u) {
        const int ub = ub0 + u;
        live[u] = ub < nub && gmem(d.rab_lo)[ub] <= ab && ab < gmem(d.rab_hi)[ub];
        first[u] = live[u] && gmem(d.rab_lo)[ub] == ab;
    }
    float gx = 0.f;
    const int n = ab * VRK_AB + i;           // B operand column (antenna) of this lane
    const bool nok = n < d.nt;
    const int per = (be0 - bs0 + kGW - 1) / kGW;
    const int bs = bs0 + w * per, be = min(be0, bs + per);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc[kUG];
#pragma unroll
    for (int u = 0; u < kUG; ++u) acc[u] = C3{z, z, z};
    constexpr int kQ = 2;   // MFMA reduction steps (4 RHS each) per iteration
    for (int b0 = bs; b0 < be; b0 += 4 * kQ) {
        float2 y[kQ], xv[kQ], v[kQ][kUG], mu[kQ][kUG];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int b = b0 + 4 * q + kk;
            const bool bok = b < be;
            y[q] = xv[q] = float2{0.f, 0.f};
            if (bok && nok) {
                const float2 gx = GX[(int64_t)b * ldgx + n], xa = XA[(int64_t)b * ldxa + n];
                y[q] = float2{gx.x - xa.x, gx.y - xa.y};
                xv[q] = X[(int64_t)b * ldx + n];
            }
#pragma unroll
            for (int u = 0; u < kUG; ++u) {
                v[q][u] = mu[q][u] = float2{0.f, 0.f};
                if (live[u] && bok) {
                    const int64_t o = (int64_t)b * kpad + (ub0 + u) * VRK_UB + i;
                    v[q][u] = VS[o];
                    mu[q][u] = MS[o];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const float2 cy = float2{y[q].x, -y[q].y}, cx_ = float2{xv[q].x, -xv[q].y};
#pragma unroll
            for (int u = 0; u < kUG; ++u) {
                if (first[u]) gx += mu[q][u].x * v[q][u].x + mu[q][u].y * v[q][u].y;
                if (live[u]) {
                    c3mfma(acc[u], v[q][u], cy);                                  // v conj(y)
                    c3mfma(acc[u], float2{-mu[q][u].x, -mu[q][u].y}, cx_);        // - mu conj(x)
                }
            }
        }
    }
    // D layout: lane (j, g) register r holds user 4 g + r, antenna j
    const int jj = lane & 15, gg = lane >> 4;
#pragma unroll
    for (int u = 0; u < kUG; ++u) {
        const f4 re = acc[u].u - acc[u].v, im = acc[u].w - acc[u].u - acc[u].v;
#pragma unroll
        for (int r = 0; r < 4; ++r) part[w][u][(4 * gg + r) * 16 + jj] = float2{re[r], im[r]};
    }
    __syncthreads();
    // thread tid owns entry tid of every block: user tid / 16, antenna tid % 16
    const int ii = tid >> 4, nj = tid & 15, nn = ab * VRK_AB + nj;
#pragma unroll
    for (int u = 0; u < kUG; ++u) {
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int ww = 0; ww < kGW; ++ww) {
            sr += part[ww][u][tid].x;
            si += part[ww][u][tid].y;
        }
        if (out) {
            out[u * 256 + tid] = float2{sr, si};   // partial over this workgroup's RHS range
        } else if (live[u]) {
            const int kq = (ub0 + u) * VRK_UB + ii;
            if (kq < d.k) {
                const int us = gmem(d.perm)[kq];
                if (nn >= gmem(d.vs)[us] && nn < gmem(d.ve)[us])
                    gmem(static_cast<float2 *>(d.GH))[(int64_t)us * d.ldgh + nn] = float2{sr, si};
            }
        }
    }
    return gx;
}

// Workgroup (tile, u): sum the RHS-split partials of user block 4 ubg + u of
// the tile in fixed order and write its VR band entries of GH (nsplit > 1).
// Workgroup (first tile of a problem, 0) also adds the gxi partials of its
// problem's tiles.
__global__ void __launch_bounds__(256) k_adj_grads_reduce(const VrkDesc *descs, const int4 *tiles, int nsplit,
                                                          const float2 *gpart, const float *gxpart)
{
    const int4 tl = gmem(tiles)[blockIdx.x];
    CDesc &d = ((CDesc *)descs)[__builtin_amdgcn_readfirstlane(tl.x)];
    const int tid = threadIdx.x, u = blockIdx.y;
    const int flags = __builtin_amdgcn_readfirstlane(tl.w);
    if ((flags & 1) && u == 0 && tid < 64) {
        // this problem's tiles: blockIdx.x and the next (flags >> 2) - 1
        const int64_t n = (int64_t)(flags >> 2) * nsplit, e0 = (int64_t)blockIdx.x * nsplit;
        float t = 0.f;
        for (int64_t e = tid; e < n; e += 64) t += gmem(gxpart)[e0 + e];
        t = wave_sum(t);
        if (tid == 0) *gmem(d.gxi) = -(double)t;
    }
    if (nsplit <= 1 || tl.y < 0) return;
    const int ub = __builtin_amdgcn_readfirstlane(tl.y) * kUG + u, ab = __builtin_amdgcn_readfirstlane(tl.z);
    if (ub >= d.nub || ab < gmem(d.rab_lo)[ub] || ab >= gmem(d.rab_hi)[ub]) return;
    const int ii = tid >> 4, nj = tid & 15, nn = ab * VRK_AB + nj;
    const gp<const float2> src = gmem(gpart) + (int64_t)blockIdx.x * nsplit * kUG * 256 + u * 256 + tid;
    float sr = 0.f, si = 0.f;
#pragma unroll 8
    for (int sp = 0; sp < nsplit; ++sp) {
        const float2 p = src[(int64_t)sp * kUG * 256];
        sr += p.x;
        si += p.y;
    }
    const int kq = ub * VRK_UB + ii;
    if (kq < d.k) {
        const int us = gmem(d.perm)[kq];
        if (nn >= gmem(d.vs)[us] && nn < gmem(d.ve)[us])
            gmem(static_cast<float2 *>(d.GH))[(int64_t)us * d.ldgh + nn] = float2{sr, si};
    }
}

// Workgroup (tile, split): one RHS range of a tile; with nsplit 1 it writes
// GH directly, else its partials to gpart. Every workgroup writes its share
// of sum_{b,k} conj(mu) v (dL/dxi is minus its real part) to gxpart: the
// users of the blocks whose first antenna block is the tile's, over its RHS
// range, from the v and mu it loads anyway.
__global__ void __launch_bounds__(kGW * 64) k_adj_grads_mfma(const VrkDesc *descs, const int4 *tiles, int nsplit,
                                                             float2 *gpart, float *gxpart)
{
    __shared__ float2 part[kGW][kUG][256];
    __shared__ float red[kGW];
    const int tix = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    const int4 tl = gmem(tiles)[tix];   // (problem, user-block group, antenna block, flags)
    CDesc &d = ((CDesc *)descs)[__builtin_amdgcn_readfirstlane(tl.x)];
    const int ubg = __builtin_amdgcn_readfirstlane(tl.y), ab = __builtin_amdgcn_readfirstlane(tl.z);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int B = d.nrhs;
    const int per = (B + nsplit - 1) / nsplit;
    const int bs0 = min(B, split * per), be0 = min(B, bs0 + per);
    // the workgroup's share of sum conj(mu) v (dL/dxi = -Re of the total)
    float acc = 0.f;
    if (ubg >= 0)
        acc = grads_group(d, ubg, ab, bs0, be0, part,
                          nsplit > 1 ? gmem(gpart) + ((int64_t)tix * nsplit + split) * kUG * 256 : nullptr);
    acc = wave_sum(acc);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (tid == 0) {
        float t = 0.f;
        for (int q = 0; q < kGW; ++q) t += red[q];
        gmem(gxpart)[blockIdx.x] = t;
    }
}


}  // namespace

hipError_t vrk_launch_adjoint_grads_mfma(const VrkDesc *desc, const int4 *tiles, int32_t ntiles, int32_t nsplit,
                                         float2 *gpart, float *gxpart, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_grads_mfma, dim3((unsigned)ntiles * nsplit), dim3(kGW * 64), 0, s, desc, tiles, nsplit,
                       gpart, gxpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_grads_reduce, dim3(ntiles, kUG), dim3(256), 0, s, desc, tiles, nsplit, gpart, gxpart);
    return hipGetLastError();
}
