// Adjoint (implicit differentiation) gradient products of the MFMA engine,
// complex64.
//
// For x = H^H v with v = (H H^H + xi I)^-1 s, an incoming gradient
// g = 2 dL/d conj(x) and mu = (H H^H + xi I)^-1 H g from the adjoint solve:
//   GH = sum_b v_b (g_b - H^H mu_b)^H - mu_b x_b^H     on the VR band entries
//   gxi = -Re sum_b mu_b^H v_b
// Since x_b = H^H v_b, both products with an x reduce to the K x K matrix
// C = sum_b v_b mu_b^H:
//   GH = sum_b v_b g_b^H - (C + C^H) H,   gxi = -Re tr C,
// and C is needed only on the Gram block pattern (a band entry (k, n) meets
// H[k', n] != 0 only for users k' whose VR overlaps that of k). Two
// kernels: the RHS-split partials of the blocks of C together with those of
// the band tiles of sum_b v_b g_b^H, then per band tile the fixed-order sum
// of its splits minus (C + C^H) H, and dL/dxi. All products run on
// v_mfma_f32_16x16x4f32.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

using CDesc = const VRK_CONST VrkDesc;
template <typename T>
using gp = VRK_GLOBAL T *;

// Blocks of C: workgroup (problem, block p = (ub, ub'), split) sums
// v_b[16 ub + i] conj(mu_b[16 ub' + j]) over its share of the RHS; the range
// is split over the waves and reduced through LDS in fixed order, and the
// partial goes to Cblk[p][split].
constexpr int kGW = 4;
constexpr int kUG = VRK_GRAD_UG;
constexpr int kCQ = 8;          // reduction steps (4 RHS each) per batch of loads
constexpr int kMaxCsplit = 4;   // RHS splits of a C block at most

__device__ __forceinline__ void cmat_part(CDesc &d, int p, int ub, int split, int csplit, float2 (*part)[256])
{
    const int ubc = __builtin_amdgcn_readfirstlane(gmem(d.cp_col)[p]);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 15, kk = lane >> 4;
    const int B = d.nrhs, kpad = d.nub * VRK_UB;
    const int per = (B + csplit - 1) / csplit;
    const int bs0 = min(B, split * per), be0 = min(B, bs0 + per);
    const int pw = (be0 - bs0 + kGW - 1) / kGW;
    const int bs = bs0 + w * pw, be = min(be0, bs + pw);
    // A operand: v of user 16 ub + i; B operand: conj(mu) of user 16 ub' + i
    const gp<const float2> VS = gmem(static_cast<const float2 *>(d.Vsrt)) + VRK_UB * ub + i;
    const gp<const float2> MS = gmem(static_cast<const float2 *>(d.Msrt)) + VRK_UB * ubc + i;
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc = {z, z, z};
    for (int b0 = bs; b0 < be; b0 += 4 * kCQ) {
        float2 a[kCQ], m[kCQ];
#pragma unroll
        for (int q = 0; q < kCQ; ++q) {
            const int b = b0 + 4 * q + kk;
            a[q] = m[q] = float2{0.f, 0.f};
            if (b < be) {
                a[q] = VS[(int64_t)b * kpad];
                m[q] = MS[(int64_t)b * kpad];
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
        for (int q = 0; q < kCQ; ++q) c3mfma(acc, a[q], float2{m[q].x, -m[q].y});
    }
    // D layout: lane (j, g) register r holds row 4 g + r, column j
    const int jj = lane & 15, gg = lane >> 4;
    const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
#pragma unroll
    for (int r = 0; r < 4; ++r) part[w][(4 * gg + r) * 16 + jj] = float2{re[r], im[r]};
    __syncthreads();
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int ww = 0; ww < kGW; ++ww) {
        sr += part[ww][tid].x;
        si += part[ww][tid].y;
    }
    gmem(static_cast<float2 *>(d.Cblk))[((int64_t)p * csplit + split) * 256 + tid] = float2{sr, si};
}

// GH on the band tiles (ub, ab) of the user blocks ub = 4 ubg .. 4 ubg + 3
// that meet antenna block ab: D[user i][antenna j] = sum_b v_b[i] conj(g_b[j])
// (A = V^T, B = conj(GX)) over an RHS range. A wave loads the antenna
// operands of 4 RHS once for all blocks of the group; v comes from the
// VR-start-order copy (16 users = 128 contiguous bytes). The range is split
// over the waves and reduced through LDS; the sum goes to GH (out null) or
// to a partial.
constexpr int kQ = 4;   // reduction steps (4 RHS each) per batch of loads

// The whole stages of one wave's RHS range [bs, be) for the band tile
// blocks in MASK (bit u: block ub0 + u meets the antenna block; a
// compile-time set, so every load is unconditional and the compiler knows
// how many are in flight): a stage is KP steps of 4 RHS, the next stage's
// loads are issued before this stage's products. After the last stage the
// pointers stop advancing, so the loads of the stage after it repeat the
// last one (in range) and are not used. Returns the first RHS not done.
template <int MASK>
__device__ __forceinline__ int band_stages(gp<const float2> gy, gp<const float2> gv, int64_t ldgx, int kpad, int bs,
                                           int be, C3 (&acc)[kUG])
{
    constexpr int nl = __builtin_popcount(MASK);
    constexpr int KP = nl <= 2 ? 4 : 2;
    const int64_t sy = 4 * ldgx, sv = 4 * (int64_t)kpad;
    const int nst = (be - bs) / (4 * KP);
    if (nst <= 0) return bs;
    struct Stage {
        float2 y[KP], v[KP][kUG];
    };
    auto load = [&](Stage &t) {
#pragma unroll
        for (int q = 0; q < KP; ++q) t.y[q] = gy[q * sy];
#pragma unroll
        for (int u = 0; u < kUG; ++u)
            if (MASK >> u & 1) {
#pragma unroll
                for (int q = 0; q < KP; ++q) t.v[q][u] = gv[q * sv + u * VRK_UB];
            }
    };
    auto advance = [&](bool more) {
        gy += more ? KP * sy : 0;
        gv += more ? KP * sv : 0;
    };
    auto mul = [&](const Stage &t) {
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const float2 cy = float2{t.y[q].x, -t.y[q].y};
#pragma unroll
            for (int u = 0; u < kUG; ++u)
                if (MASK >> u & 1) c3mfma(acc[u], t.v[q][u], cy);
        }
    };
    Stage A, B;
    load(A);
#pragma unroll 1
    for (int st = 0; st < nst; st += 2) {
        advance(st + 1 < nst);
        load(B);   // stage st + 1, or stage st again
        __builtin_amdgcn_sched_barrier(0);   // the loads issue before the products
        mul(A);    // stage st
        advance(st + 2 < nst);
        load(A);   // stage st + 2, or the last stage again
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < nst) mul(B);
    }
    return bs + nst * 4 * KP;
}

__device__ __forceinline__ void grads_group(CDesc &d, int ubg, int ab, int bs0, int be0, float2 (*part)[kUG][256],
                                            gp<float2> out)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 15, kk = lane >> 4;
    const gp<const float2> VS = gmem(static_cast<const float2 *>(d.Vsrt));
    const gp<const float2> GX = gmem(static_cast<const float2 *>(d.GX));
    const int64_t ldgx = d.ldgx;
    const int nub = d.nub, kpad = nub * VRK_UB;
    const int ub0 = ubg * kUG;
    // blocks of the group that meet ab (wave-uniform)
    bool live[kUG];
#pragma unroll
    for (int u = 0; u < kUG; ++u) {
        const int ub = ub0 + u;
        live[u] = ub < nub && gmem(d.rab_lo)[ub] <= ab && ab < gmem(d.rab_hi)[ub];
    }
    const int n = ab * VRK_AB + i;           // B operand column (antenna) of this lane
    const bool nok = n < d.nt;
    const int per = (be0 - bs0 + kGW - 1) / kGW;
    const int bs = bs0 + w * per, be = min(be0, bs + per);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    C3 acc[kUG];
#pragma unroll
    for (int u = 0; u < kUG; ++u) acc[u] = C3{z, z, z};
    // whole stages: every RHS of the stage is in range, so the loads need no
    // per-lane guard; the antenna operand comes from a clamped column (a
    // column past nt only feeds output entries that are never written)
    int b0 = bs;
    {
        int mask = 0;
#pragma unroll
        for (int u = 0; u < kUG; ++u) mask |= live[u] ? 1 << u : 0;
        mask = __builtin_amdgcn_readfirstlane(mask);
        gp<const float2> gy = GX + (int64_t)(bs + kk) * ldgx + (nok ? n : d.nt - 1);
        gp<const float2> gv = VS + (int64_t)(bs + kk) * kpad + ub0 * VRK_UB + i;
        switch (mask) {
#define VRK_BAND_CASE(M) \
    case M: b0 = band_stages<M>(gy, gv, ldgx, kpad, bs, be, acc); break;
            VRK_BAND_CASE(1) VRK_BAND_CASE(2) VRK_BAND_CASE(3) VRK_BAND_CASE(4) VRK_BAND_CASE(5)
            VRK_BAND_CASE(6) VRK_BAND_CASE(7) VRK_BAND_CASE(8) VRK_BAND_CASE(9) VRK_BAND_CASE(10)
            VRK_BAND_CASE(11) VRK_BAND_CASE(12) VRK_BAND_CASE(13) VRK_BAND_CASE(14) VRK_BAND_CASE(15)
#undef VRK_BAND_CASE
            default: break;
        }
    }
    // the last partial batch, guarded per lane
    for (; b0 < be; b0 += 4 * kQ) {
        float2 y[kQ], v[kQ][kUG];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int b = b0 + 4 * q + kk;
            const bool bok = b < be;
            y[q] = float2{0.f, 0.f};
            if (bok && nok) y[q] = GX[(int64_t)b * ldgx + n];
#pragma unroll
            for (int u = 0; u < kUG; ++u) {
                v[q][u] = float2{0.f, 0.f};
                if (live[u] && bok) v[q][u] = VS[(int64_t)b * kpad + (ub0 + u) * VRK_UB + i];
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const float2 cy = float2{y[q].x, -y[q].y};
#pragma unroll
            for (int u = 0; u < kUG; ++u)
                if (live[u]) c3mfma(acc[u], v[q][u], cy);
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
}

// Workgroups [0, nctile): the C blocks (problem, block, split, row block);
// then (band tile, split): one RHS range of a band tile, written to GH with
// nsplit 1, else to its partial in gpart. The band workgroups take the
// tiles in the order `order` lists them (the groups of one antenna block
// side by side), dealt out so that each XCD (workgroup x runs on XCD x % 8)
// walks a contiguous run of that list: tiles that read the same columns of
// the incoming gradient run together on one L2. Four waves per SIMD (left
// alone, the compiler takes a third more registers and three).
__global__ void __launch_bounds__(kGW * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_adj_grads_mfma(const VrkDesc *descs, const int4 *tiles, const int32_t *order, int ntiles, int nsplit,
                 const int4 *ctiles, int nctile, int csplit, float2 *gpart)
{
    __shared__ float2 part[kGW][kUG][256];
    if ((int)blockIdx.x < nctile) {
        const int4 tl = gmem(ctiles)[blockIdx.x];
        CDesc &d = ((CDesc *)descs)[__builtin_amdgcn_readfirstlane(tl.x)];
        cmat_part(d, __builtin_amdgcn_readfirstlane(tl.y), __builtin_amdgcn_readfirstlane(tl.w),
                  __builtin_amdgcn_readfirstlane(tl.z), csplit, part[0]);
        return;
    }
    const int item = xcd_item(blockIdx.x - nctile, ntiles * nsplit);
    const int tix = gmem(order)[item / nsplit], split = item % nsplit;
    const int4 tl = gmem(tiles)[tix];   // (problem, user-block group, antenna block, flags)
    CDesc &d = ((CDesc *)descs)[__builtin_amdgcn_readfirstlane(tl.x)];
    const int ubg = __builtin_amdgcn_readfirstlane(tl.y), ab = __builtin_amdgcn_readfirstlane(tl.z);
    if (ubg < 0) return;
    const int B = d.nrhs;
    const int per = (B + nsplit - 1) / nsplit;
    const int bs0 = min(B, split * per), be0 = min(B, bs0 + per);
    grads_group(d, ubg, ab, bs0, be0, part,
                nsplit > 1 ? gmem(gpart) + ((int64_t)tix * nsplit + split) * kUG * 256 : nullptr);
}

// Workgroup (run of consecutive band tiles of one user-block group), wave u:
// user block ub = 4 ubg + u on the antenna blocks ab of the run's tiles. Per
// tile its entries start from the sum of the RHS-split partials in fixed
// order (nsplit > 1) or from GH; then acc -= (C + C^H)[block ub, :]
// H[:, block ab] as an MFMA product over the column blocks ub' of ub whose
// bands meet ab, with A[i][k] = -(C + C^H) entry (16 ub + i, 16 ub' + k) (C
// summed over its splits; kRP blocks held in registers per pass over the
// run) and B[k][j] = H of user 16 ub' + k at antenna 16 ab + j from the
// residual tiles of ub' (zero off the VRs); the result goes to the VR band
// entries of GH. Wave 0 of a problem's first run also writes
// dL/dxi = -Re tr C.
constexpr int kRP = 4;

__global__ void __launch_bounds__(kGW * 64) __attribute__((amdgpu_waves_per_eu(4))) k_adj_grads_reduce(const VrkDesc *descs, const int4 *tiles,
                                                             const int4 *runs, int nsplit, int csplit,
                                                             const float2 *gpart)
{
    // each XCD takes a contiguous run of the list (neighbouring runs read the same tiles of H)
    const int4 rn = gmem(runs)[xcd_item(blockIdx.x, gridDim.x)];   // (first tile, tile count, flags, 0)
    const int t0 = __builtin_amdgcn_readfirstlane(rn.x), nt = __builtin_amdgcn_readfirstlane(rn.y);
    const int4 tl0 = gmem(tiles)[t0];
    CDesc &d = ((CDesc *)descs)[__builtin_amdgcn_readfirstlane(tl0.x)];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
    const gp<const float2> CB = gmem(static_cast<const float2 *>(d.Cblk));
    if ((__builtin_amdgcn_readfirstlane(rn.z) & 1) && w == 0) {
        float t = 0.f;
        for (int e = lane; e < d.nub * VRK_UB; e += 64) {
            const int64_t p = gmem(d.cp_diag)[e >> 4];
            for (int cs = 0; cs < csplit; ++cs) t += CB[(p * csplit + cs) * 256 + (e & 15) * 17].x;
        }
        t = wave_sum(t);
        if (lane == 0) *gmem(d.gxi) = -(double)t;
    }
    const int ubg = __builtin_amdgcn_readfirstlane(tl0.y);
    if (ubg < 0) return;
    const int ub = ubg * kUG + w;
    if (ub >= d.nub) return;
    const int lo_ub = gmem(d.rab_lo)[ub], hi_ub = gmem(d.rab_hi)[ub];
    // this lane's entries: user 16 ub + 4 g + r, antenna 16 ab + j (D layout)
    const int j = i, g = kk;
    int us[4], vs[4], ve[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int kq = ub * VRK_UB + 4 * g + r;
        us[r] = -1;
        vs[r] = ve[r] = 0;
        if (kq < d.k) {
            us[r] = gmem(d.perm)[kq];
            vs[r] = gmem(d.vs)[us[r]];
            ve[r] = gmem(d.ve)[us[r]];
        }
    }
    const gp<float2> GH = gmem(static_cast<float2 *>(d.GH));
    const gp<const float2> HA = gmem(static_cast<const float2 *>(d.HA));
    const int p0 = __builtin_amdgcn_readfirstlane(gmem(d.cp_off)[ub]);
    const int p1 = __builtin_amdgcn_readfirstlane(gmem(d.cp_off)[ub + 1]);
#pragma unroll 1
    for (int pb = p0; pb < p1; pb += kRP) {
        // A operands of this pass's blocks, one RHS split of all of them at a time
        float2 A[kRP][4];
        int lo[kRP], hi[kRP], pc[kRP], pt[kRP];
        int64_t hoff[kRP];
#pragma unroll
        for (int q = 0; q < kRP; ++q) {
            const int p = min(pb + q, p1 - 1);
            const int ubc = __builtin_amdgcn_readfirstlane(gmem(d.cp_col)[p]);
            pc[q] = p;
            pt[q] = __builtin_amdgcn_readfirstlane(gmem(d.cp_tr)[p]);
            lo[q] = __builtin_amdgcn_readfirstlane(gmem(d.rab_lo)[ubc]);
            hi[q] = __builtin_amdgcn_readfirstlane(gmem(d.rab_hi)[ubc]);
            hoff[q] = gmem(d.ha_off)[ubc];
#pragma unroll
            for (int s = 0; s < 4; ++s) A[q][s] = float2{0.f, 0.f};
        }
#pragma unroll 1
        for (int cs = 0; cs < csplit; ++cs)
#pragma unroll
            for (int q0 = 0; q0 < kRP; q0 += 2) {   // two blocks' loads at a time
                float2 c1[2][4], c2[2][4];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k = 4 * s + kk;
                        c1[q][s] = CB[((int64_t)pc[q0 + q] * csplit + cs) * 256 + i * 16 + k];
                        c2[q][s] = CB[((int64_t)pt[q0 + q] * csplit + cs) * 256 + k * 16 + i];
                    }
                __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        float2 &x = A[q0 + q][s];
                        x = float2{x.x - c1[q][s].x - c2[q][s].x, x.y - c1[q][s].y + c2[q][s].y};
                    }
            }
#pragma unroll 1
        for (int t = t0; t < t0 + nt; ++t) {
            const int ab = __builtin_amdgcn_readfirstlane(gmem(tiles)[t].z);
            if (ab < lo_ub || ab >= hi_ub) continue;
            const int nn = ab * VRK_AB + j;
            bool in[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) in[r] = us[r] >= 0 && nn >= vs[r] && nn < ve[r];
            // residual tile c of ub' holds H[16 ub' + i'][16 ab + 4 kk' + m] at
            // 64 m + i' + 16 kk' (ab = lo + c / 4, m = c % 4)
            float2 h[kRP][4];
#pragma unroll
            for (int q = 0; q < kRP; ++q) {
                const bool meets = pb + q < p1 && ab >= lo[q] && ab < hi[q];
                const gp<const float2> ht = HA + (hoff[q] + 4 * (int64_t)(ab - lo[q])) * 64;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    h[q][s] = float2{0.f, 0.f};
                    if (meets) h[q][s] = ht[64 * (i & 3) + 4 * s + kk + 16 * (i >> 2)];
                }
            }
            f4 r0, i0;
#pragma unroll
            for (int r = 0; r < 4; ++r) r0[r] = i0[r] = 0.f;
            if (pb == p0 && nsplit > 1) {
                const gp<const float2> src = gmem(gpart) + (int64_t)t * nsplit * kUG * 256 + w * 256;
#pragma unroll 4
                for (int sp = 0; sp < nsplit; ++sp)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float2 p = src[(int64_t)sp * kUG * 256 + (4 * g + r) * 16 + j];
                        r0[r] += p.x;
                        i0[r] += p.y;
                    }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (in[r]) {
                        const float2 p = GH[(int64_t)us[r] * d.ldgh + nn];
                        r0[r] = p.x;
                        i0[r] = p.y;
                    }
            }
            // C3 state with Re = u - v = r0 and Im = w - u - v = i0
            C3 acc = {r0, f4{0.f, 0.f, 0.f, 0.f}, r0 + i0};
#pragma unroll
            for (int q = 0; q < kRP; ++q)
                if (pb + q < p1 && ab >= lo[q] && ab < hi[q])
#pragma unroll
                    for (int s = 0; s < 4; ++s) c3mfma(acc, A[q][s], h[q][s]);
            const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (in[r]) GH[(int64_t)us[r] * d.ldgh + nn] = float2{re[r], im[r]};
        }
    }
}


// Tiles with RHS splits (nsplit > 1; few tiles): workgroup (band tile, u) of
// 4 waves for user block ub = 4 ubg + u, wave x taking the splits x, x + 4,
// ... and the column blocks p0 + x, p0 + x + 4, ... of the correction (as in
// k_adj_grads_reduce, C summed over its splits); the four waves are added
// through LDS in fixed order.
__global__ void __launch_bounds__(kGW * 64) k_adj_grads_reduce_split(const VrkDesc *descs, const int4 *tiles,
                                                                   int nsplit, int csplit, const float2 *gpart)
{
    __shared__ float2 part[kGW][256];
    const int4 tl = gmem(tiles)[blockIdx.x];
    CDesc &d = ((CDesc *)descs)[__builtin_amdgcn_readfirstlane(tl.x)];
    const int x = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
    const int u = blockIdx.y;
    const gp<const float2> CB = gmem(static_cast<const float2 *>(d.Cblk));
    if ((__builtin_amdgcn_readfirstlane(tl.w) & 1) && u == 0 && x == 0) {
        float t = 0.f;
        for (int e = lane; e < d.nub * VRK_UB; e += 64) {
            const int64_t p = gmem(d.cp_diag)[e >> 4];
            for (int cs = 0; cs < csplit; ++cs) t += CB[(p * csplit + cs) * 256 + (e & 15) * 17].x;
        }
        t = wave_sum(t);
        if (lane == 0) *gmem(d.gxi) = -(double)t;
    }
    const int ubg = __builtin_amdgcn_readfirstlane(tl.y);
    if (ubg < 0) return;   // the whole workgroup
    const int ub = ubg * kUG + u, ab = __builtin_amdgcn_readfirstlane(tl.z);
    if (ub >= d.nub || ab < gmem(d.rab_lo)[ub] || ab >= gmem(d.rab_hi)[ub]) return;   // the whole workgroup
    // this lane's entries: user 16 ub + 4 g + r, antenna 16 ab + j (D layout)
    const int j = i, g = kk;
    f4 r0 = {0.f, 0.f, 0.f, 0.f}, i0 = {0.f, 0.f, 0.f, 0.f};
    {
        const gp<const float2> src = gmem(gpart) + (int64_t)blockIdx.x * nsplit * kUG * 256 + u * 256;
#pragma unroll 2
        for (int sp = x; sp < nsplit; sp += kGW)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float2 p = src[(int64_t)sp * kUG * 256 + (4 * g + r) * 16 + j];
                r0[r] += p.x;
                i0[r] += p.y;
            }
    }
    C3 acc = {r0, f4{0.f, 0.f, 0.f, 0.f}, r0 + i0};
    const gp<const float2> HA = gmem(static_cast<const float2 *>(d.HA));
    const int p0 = __builtin_amdgcn_readfirstlane(gmem(d.cp_off)[ub]);
    const int p1 = __builtin_amdgcn_readfirstlane(gmem(d.cp_off)[ub + 1]);
#pragma unroll 1
    for (int p = p0 + x; p < p1; p += kGW) {
        const int ubc = __builtin_amdgcn_readfirstlane(gmem(d.cp_col)[p]);
        const int lo = __builtin_amdgcn_readfirstlane(gmem(d.rab_lo)[ubc]);
        if (ab < lo || ab >= gmem(d.rab_hi)[ubc]) continue;
        const int pt = __builtin_amdgcn_readfirstlane(gmem(d.cp_tr)[p]);
        const gp<const float2> ht = HA + (gmem(d.ha_off)[ubc] + 4 * (int64_t)(ab - lo)) * 64;
        float2 h[4], c1[kMaxCsplit][4], c2[kMaxCsplit][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + kk;
            h[s] = ht[64 * (i & 3) + k + 16 * (i >> 2)];
#pragma unroll
            for (int cs = 0; cs < kMaxCsplit; ++cs) {
                c1[cs][s] = c2[cs][s] = float2{0.f, 0.f};
                if (cs < csplit) {
                    c1[cs][s] = CB[((int64_t)p * csplit + cs) * 256 + i * 16 + k];
                    c2[cs][s] = CB[((int64_t)pt * csplit + cs) * 256 + k * 16 + i];
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int cs = 0; cs < kMaxCsplit; ++cs) {
                ar += c1[cs][s].x + c2[cs][s].x;
                ai += c1[cs][s].y - c2[cs][s].y;
            }
            c3mfma(acc, float2{-ar, -ai}, h[s]);
        }
    }
    const f4 re = acc.u - acc.v, im = acc.w - acc.u - acc.v;
#pragma unroll
    for (int r = 0; r < 4; ++r) part[x][(4 * g + r) * 16 + j] = float2{re[r], im[r]};
    __syncthreads();
    if (x != 0) return;
    const int nn = ab * VRK_AB + j;
    const gp<float2> GH = gmem(static_cast<float2 *>(d.GH));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int kq = ub * VRK_UB + 4 * g + r, e = (4 * g + r) * 16 + j;
        if (kq >= d.k) continue;
        const int us = gmem(d.perm)[kq];
        if (nn < gmem(d.vs)[us] || nn >= gmem(d.ve)[us]) continue;
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int xx = 0; xx < kGW; ++xx) {
            sr += part[xx][e].x;
            si += part[xx][e].y;
        }
        GH[(int64_t)us * d.ldgh + nn] = float2{sr, si};
    }
}


}  // namespace

hipError_t vrk_launch_adjoint_grads_mfma(const VrkDesc *desc, const int4 *tiles, const int32_t *order, int32_t ntiles,
                                         int32_t nsplit,
                                         const int4 *ctiles, int32_t nctiles, int32_t csplit, const int4 *runs,
                                         int32_t nruns, float2 *gpart, hipStream_t s)
{
    if (csplit < 1 || csplit > kMaxCsplit) return hipErrorInvalidValue;
    const int64_t nwg = (int64_t)nctiles + (int64_t)ntiles * nsplit;
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_grads_mfma, dim3((unsigned)nwg), dim3(kGW * 64), 0, s, desc, tiles, order, ntiles,
                       nsplit, ctiles, nctiles, csplit, gpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ntiles <= 0) return e;
    if (nsplit > 1)
        hipLaunchKernelGGL(k_adj_grads_reduce_split, dim3(ntiles, kUG), dim3(kGW * 64), 0, s, desc, tiles, nsplit,
                           csplit, gpart);
    else if (nruns > 0)
        hipLaunchKernelGGL(k_adj_grads_reduce, dim3(nruns), dim3(kGW * 64), 0, s, desc, tiles, runs, nsplit,
                           csplit, gpart);
    return hipGetLastError();
}
