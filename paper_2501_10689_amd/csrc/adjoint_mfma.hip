// Adjoint (implicit differentiation) products of the MFMA engine, complex64.
//
// For x = H^H (H H^H + xi I)^-1 s and an incoming gradient g = 2 dL/d conj(x):
//   b = H g                                   (right-hand side of the adjoint solve)
//   GH = sum_b v_b (g_b - xh_b)^H - mu_b x_b^H  on the VR band entries
//   gxi = -Re sum_b mu_b^H v_b
// with mu = (H H^H + xi I)^-1 H g and xh = H^H mu from the adjoint solve.
// Both products run on v_mfma_f32_16x16x4f32 over the band tiles of the plan.
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

// b = H g for one tile of 16 RHS and one 16-user block (one wave):
// D[user][rhs] = sum over the block's band chunks of HA-tile x GX.
__global__ void __launch_bounds__(64) k_adj_rhs_mfma(const VrkDesc *descs, const VrkWork *work)
{
    const VrkWork wk = work[blockIdx.x];
    const VrkDesc &d = descs[wk.prob];
    const int ub = blockIdx.y;
    if (ub >= d.nub) return;
    const int lane = threadIdx.x, j = lane & 15, g = lane >> 4;
    const int b = wk.tile * VRK_TILE_RHS + j;
    const float2 *HA = reinterpret_cast<const float2 *>(d.HA);
    const float2 *GX = reinterpret_cast<const float2 *>(d.GX);
    const int lo = d.rab_lo[ub], hi = d.rab_hi[ub];
    const int64_t hb = d.ha_off[ub];
    const bool bok = b < d.nrhs;
    const float2 *grow = GX + (int64_t)(bok ? b : 0) * d.ldgx;
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc = {z, z, z};
    for (int ab = lo; ab < hi; ++ab) {
        const float2 *hp = HA + (hb + 4 * (int64_t)(ab - lo)) * 64 + lane;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int n = 16 * ab + 4 * g + m;   // reduction slot g of chunk (ab, m)
            float2 x = (bok && n < d.nt) ? grow[n] : float2{0.f, 0.f};
            c3mfma(acc, hp[64 * m], x);
        }
    }
    const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
    if (bok) {
        float2 *out = reinterpret_cast<float2 *>(d.Sadj) + (int64_t)b * d.k;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ku = ub * VRK_UB + 4 * g + r;
            if (ku < d.k) out[d.perm[ku]] = float2{re[r], im[r]};
        }
    }
}

// GH on the band tile (ub, ab): D[user i][antenna j] = sum_b A[i][b] B[b][j]
// with A = V^T, B = conj(GX - Xadj) plus A = -GS^T, B = conj(X), the RHS
// dimension split over the 8 waves and reduced through LDS.
constexpr int kGW = 8;

__device__ __forceinline__ void grads_tile(const VrkDesc &d, int ub, int ab, int bs0, int be0,
                                           float2 (*part)[256], float2 *out)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 15, kk = lane >> 4;
    const float2 *V = reinterpret_cast<const float2 *>(d.V);
    const float2 *GS = reinterpret_cast<const float2 *>(d.GS);
    const float2 *GX = reinterpret_cast<const float2 *>(d.GX);
    const float2 *XA = reinterpret_cast<const float2 *>(d.Xadj);
    const float2 *X = reinterpret_cast<const float2 *>(d.X);
    const int ku = ub * VRK_UB + i;          // A operand row (user) of this lane
    const int user = ku < d.k ? d.perm[ku] : -1;
    const int n = ab * VRK_AB + i;           // B operand column (antenna) of this lane
    const bool nok = n < d.nt;
    // this workgroup's RHS range [bs0, be0), split over the waves
    const int per = (be0 - bs0 + kGW - 1) / kGW;
    const int bs = bs0 + w * per, be = min(be0, bs + per);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc = {z, z, z};
    for (int b0 = bs; b0 < be; b0 += 4) {
        const int b = b0 + kk;
        float2 v = {0.f, 0.f}, mu = {0.f, 0.f}, y = {0.f, 0.f}, xv = {0.f, 0.f};
        if (b < be) {
            if (user >= 0) {
                v = V[(int64_t)b * d.ldv + user];
                mu = GS[(int64_t)b * d.ldgs + user];
            }
            if (nok) {
                float2 gx = GX[(int64_t)b * d.ldgx + n], xa = XA[(int64_t)b * d.nt + n];
                y = float2{gx.x - xa.x, gx.y - xa.y};
                xv = X[(int64_t)b * d.ldx + n];
            }
        }
        c3mfma(acc, v, float2{y.x, -y.y});            // v conj(y)
        c3mfma(acc, float2{-mu.x, -mu.y}, float2{xv.x, -xv.y});   // - mu conj(x)
    }
    const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
    // D layout: lane (j, g) register r holds user 4 g + r, antenna j
    const int jj = lane & 15, gg = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) part[w][(4 * gg + r) * 16 + jj] = float2{re[r], im[r]};
    __syncthreads();
    if (tid < 256) {
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int ww = 0; ww < kGW; ++ww) {
            sr += part[ww][tid].x;
            si += part[ww][tid].y;
        }
        if (out) {
            out[tid] = float2{sr, si};   // partial over this workgroup's RHS range
        } else {
            const int ii = tid >> 4, nj = tid & 15;
            const int kq = ub * VRK_UB + ii, nn = ab * VRK_AB + nj;
            if (kq < d.k) {
                const int u = d.perm[kq];
                if (nn >= d.vs[u] && nn < d.ve[u])
                    reinterpret_cast<float2 *>(d.GH)[(int64_t)u * d.ldgh + nn] = float2{sr, si};
            }
        }
    }
}

// Sum the RHS-split partials of each band tile in fixed order and write the
// VR band entries of GH.
__global__ void __launch_bounds__(256) k_adj_grads_reduce(const VrkDesc *descs, const int4 *tiles, int nsplit,
                                                          const float2 *gpart)
{
    const int4 tl = tiles[blockIdx.x];
    if (tl.y < 0) return;
    const VrkDesc &d = descs[tl.x];
    const int tid = threadIdx.x, ii = tid >> 4, nj = tid & 15;
    float sr = 0.f, si = 0.f;
    for (int sp = 0; sp < nsplit; ++sp) {
        float2 p = gpart[((int64_t)blockIdx.x * nsplit + sp) * 256 + tid];
        sr += p.x;
        si += p.y;
    }
    const int kq = tl.y * VRK_UB + ii, nn = tl.z * VRK_AB + nj;
    if (kq < d.k) {
        const int u = d.perm[kq];
        if (nn >= d.vs[u] && nn < d.ve[u])
            reinterpret_cast<float2 *>(d.GH)[(int64_t)u * d.ldgh + nn] = float2{sr, si};
    }
}

// Workgroup (tile, split): RHS range split of the band tile; with nsplit 1
// it writes GH directly, else its partial to gpart.
__global__ void __launch_bounds__(kGW * 64) k_adj_grads_mfma(const VrkDesc *descs, const int4 *tiles, int nsplit,
                                                             float2 *gpart)
{
    __shared__ float2 part[kGW][256];
    __shared__ float red[kGW];
    const int tix = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    const int4 tl = tiles[tix];   // (problem, user block, antenna block, first-of-problem)
    const VrkDesc &d = descs[tl.x];
    const int ub = tl.y, ab = tl.z;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const float2 *V = reinterpret_cast<const float2 *>(d.V);
    const float2 *GS = reinterpret_cast<const float2 *>(d.GS);
    const int B = d.nrhs;
    const int per = (B + nsplit - 1) / nsplit;
    const int bs0 = min(B, split * per), be0 = min(B, bs0 + per);
    if (ub >= 0)
        grads_tile(d, ub, ab, bs0, be0, part,
                   nsplit > 1 ? gpart + ((int64_t)tix * nsplit + split) * 256 : nullptr);
    // dL/dxi = -Re sum_{b,k} conj(mu) v, by one entry per problem
    if (tl.w && split == 0) {
        float acc = 0.f;
        const int64_t tot = (int64_t)B * d.k;
        for (int64_t e = tid; e < tot; e += kGW * 64) {
            const int b = (int)(e / d.k), k = (int)(e % d.k);
            float2 mu = GS[(int64_t)b * d.ldgs + k], v = V[(int64_t)b * d.ldv + k];
            acc += mu.x * v.x + mu.y * v.y;
        }
        acc = wave_sum(acc);
        if (lane == 0) red[w] = acc;
        __syncthreads();
        if (tid == 0) {
            float t = 0.f;
            for (int q = 0; q < kGW; ++q) t += red[q];
            *d.gxi = -(double)t;
        }
    }
}


}  // namespace

hipError_t vrk_launch_adjoint_rhs_mfma(const VrkDesc *desc, const VrkWork *work, int32_t nwork,
                                       int32_t max_nub, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_rhs_mfma, dim3(nwork, max_nub), dim3(64), 0, s, desc, work);
    return hipGetLastError();
}

hipError_t vrk_launch_adjoint_grads_mfma(const VrkDesc *desc, const int4 *tiles, int32_t ntiles, int32_t nsplit,
                                         float2 *gpart, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_grads_mfma, dim3((unsigned)ntiles * nsplit), dim3(kGW * 64), 0, s, desc, tiles, nsplit,
                       gpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit <= 1) return e;
    hipLaunchKernelGGL(k_adj_grads_reduce, dim3(ntiles), dim3(256), 0, s, desc, tiles, nsplit, gpart);
    return hipGetLastError();
}
