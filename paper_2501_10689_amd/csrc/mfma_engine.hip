// MFMA engine: 16 right-hand sides per workgroup share H; the banded
// complex products of every Kaczmarz variant run on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32, complex product as four real products).
//
// Layout. Lane l of a wave is (j, g) = (l % 16, l / 16): RHS column j and
// row group g. The iterate x of the tile never leaves registers: wave w
// owns the 16-antenna blocks ab = w + W a, and lane (j, g) holds
// x[16 ab + 4 g + r][j] in register r of float4 pair xr[a], xq[a] - the
// layout of an MFMA result tile. Feeding the residual product
//   R[u][j] = sum_n H[u][n] x[n][j]
// the reduction index of chunk (ab, m) is ordered as antenna 16 ab + 4 kk + m
// for slot kk, so register m of xr[a] is already the B operand; the packed
// residual tile (ub, ab, m) holds H of 16 users at those antennas. The
// aggregation product P[n][j] = sum_u conj(H[u][n]) phi[u][j] produces
// tiles in the same layout as x, so x += gamma P is register-local.
// Users are processed in VR-start order (perm), which keeps the nonzero
// tiles of the banded H few.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Complex product A * B accumulated with three real products (Gauss):
// u += Ar Br, v += Ai Bi, w += (Ar + Ai)(Br + Bi); then Re = u - v and
// Im = w - u - v. Operands are held one complex value per lane.
struct C3 {
    f4 u, v, w;
};

__device__ __forceinline__ C3 c3_zero()
{
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    return C3{z, z, z};
}

__device__ __forceinline__ void c3mfma(C3 &acc, float2 a, float2 b)
{
    acc.u = mfma(a.x, b.x, acc.u);
    acc.v = mfma(a.y, b.y, acc.v);
    acc.w = mfma(a.x + a.y, b.x + b.y, acc.w);
}

__device__ __forceinline__ void c3_get(const C3 &acc, f4 &re, f4 &im)
{
    re = acc.u - acc.v;
    im = acc.w - acc.u - acc.v;
}

struct MfmaLds {
    float2 *R, *Q, *Rp;
    float *nrm, *pre, *red, *snorm, *rel, *gre, *gim, *num, *phin, *pnw;
    int *posl, *active, *iters, *flags, *pick, *any;
    int *agoff, *rlo, *rhi, *hoff, *gmoff;   // copies of the tile tables of this problem
};

__host__ __device__ inline size_t mfma_lds_layout(int kpad, int nab, int W, char *base, MfmaLds *L)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 15) & ~size_t(15);
        return base ? base + o : nullptr;
    };
    char *R = take((size_t)kpad * 16 * 8);
    char *Q = take((size_t)kpad * 16 * 8);
    char *Rp = take((size_t)W * VRK_RGROUP * 16 * 8);
    char *nrm = take((size_t)kpad * 4);
    char *pre = take((size_t)W * kpad * 4);
    char *red = take((size_t)(W * 16 + 16) * 4);
    char *sc = take(16 * 4 * 8);
    char *pnw = take((size_t)W * 16 * 4);
    char *posl = take((size_t)kpad * 4);
    char *ints = take(16 * 4 * 4 + 16);
    char *tabs = take((size_t)(nab + 1 + 4 * (kpad / 16) + 1) * 4);
    if (L) {
        int *tb = (int *)tabs;
        L->agoff = tb;
        L->rlo = tb + nab + 1;
        L->rhi = L->rlo + kpad / 16;
        L->hoff = L->rhi + kpad / 16;
        L->gmoff = L->hoff + kpad / 16;
        L->R = (float2 *)R;
        L->Q = (float2 *)Q;
        L->Rp = (float2 *)Rp;
        L->nrm = (float *)nrm;
        L->pre = (float *)pre;
        L->red = (float *)red;
        float *s = (float *)sc;
        L->snorm = s;
        L->rel = s + 16;
        L->gre = s + 32;
        L->gim = s + 48;
        L->num = s + 64;
        L->phin = s + 80;
        L->pnw = (float *)pnw;
        L->posl = (int *)posl;
        int *ip = (int *)ints;
        L->active = ip;
        L->iters = ip + 16;
        L->flags = ip + 32;
        L->pick = ip + 48;
        L->any = ip + 64;
    }
    return off;
}

// Sum over the threads of each RHS column j = tid % 16; every thread gets
// its column's total. Deterministic order.
template <int W>
__device__ __forceinline__ float col_sum(float v, float *red)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    __syncthreads();
    if (lane < 16) red[w * 16 + lane] = v;
    __syncthreads();
    if (tid < 16) {
        float s = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) s += red[i * 16 + tid];
        red[W * 16 + tid] = s;
    }
    __syncthreads();
    return red[W * 16 + (tid & 15)];
}

// Per-tile constants shared by the phases below (passed by value so that
// everything stays in registers after inlining).
struct TileCtx {
    const VrkDesc *d;
    MfmaLds L;
    const float2 *S, *H, *HA, *HG, *GM;
    float2 *Xw;   // global-iterate mode: this tile's x, [ab][r][lane] (MFMA result order)
    int64_t lds;
    int K, N, nub, kpad, nab, b0, nrhs, prob;
    float xi;
};

// R <- s - H x - xi q (rows in VR-start order), two 16-user blocks at a time
// with a deterministic cross-wave reduction through LDS. With `ogrk` only
// the rows of X_pick are written (the others keep their value, Theorem 2).
template <int W, int NA>
__device__ __forceinline__ void tile_residual(const TileCtx &c, const f4 (&xr)[NA ? NA : 1],
                                              const f4 (&xq)[NA ? NA : 1], bool ogrk)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, j = lane & 15, g = lane >> 4;
    const VrkDesc &d = *c.d;
    const int nug = (c.nub + 1) / 2;
    const int er = tid >> 4, rows_per_pass = W * 4;
#pragma unroll 1
    for (int gi = 0; gi < nug; ++gi) {
#pragma unroll 1
        for (int u2 = 0; u2 < 2; ++u2) {
            const int ub = gi * 2 + u2;
            C3 acc = c3_zero();
            if (ub < c.nub) {
                const int lo = c.L.rlo[ub], hi = c.L.rhi[ub];
                const int64_t hb = c.L.hoff[ub];
                if constexpr (NA == 0) {
                    // global iterate: the wave's blocks w, w + W, ... inside [lo, hi)
                    int ab = lo + ((w - lo) % W + W) % W;
#pragma unroll 1
                    for (; ab < hi; ab += W) {
                        const float2 *hp = c.HA + (hb + 4 * (int64_t)(ab - lo)) * 64 + lane;
                        const float2 *xp = c.Xw + (int64_t)ab * 256 + lane;
                        float2 h0 = hp[0], h1 = hp[64], h2 = hp[128], h3 = hp[192];
                        float2 x0 = xp[0], x1 = xp[64], x2 = xp[128], x3 = xp[192];
                        c3mfma(acc, h0, x0);
                        c3mfma(acc, h1, x1);
                        c3mfma(acc, h2, x2);
                        c3mfma(acc, h3, x3);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < NA; ++t) {
                        const int ab = w + W * t;
                        if (ab >= lo && ab < hi) {
                            const float2 *hp = c.HA + (hb + 4 * (int64_t)(ab - lo)) * 64 + lane;
                            float2 h0 = hp[0], h1 = hp[64], h2 = hp[128], h3 = hp[192];
                            c3mfma(acc, h0, float2{xr[t][0], xq[t][0]});
                            c3mfma(acc, h1, float2{xr[t][1], xq[t][1]});
                            c3mfma(acc, h2, float2{xr[t][2], xq[t][2]});
                            c3mfma(acc, h3, float2{xr[t][3], xq[t][3]});
                        }
                    }
                }
            }
            f4 are, aim;
            c3_get(acc, are, aim);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                c.L.Rp[(w * VRK_RGROUP + u2 * 16 + 4 * g + r) * 16 + j] = float2{are[r], aim[r]};
        }
        __syncthreads();
        for (int uu = er; uu < VRK_RGROUP; uu += rows_per_pass) {
            const int ku = gi * VRK_RGROUP + uu;
            if (ku < c.kpad) {
                float sr = 0.f, si = 0.f;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    float2 p = c.L.Rp[(ww * VRK_RGROUP + uu) * 16 + j];
                    sr += p.x;
                    si += p.y;
                }
                bool keep = true;
                if (ogrk) {
                    const int pk = c.L.pick[j];
                    if (ku < c.K && pk >= 0) {
                        const int u = d.perm[ku];
                        keep = (u == pk) || (max(d.vs[u], d.vs[pk]) < min(d.ve[u], d.ve[pk]));
                    } else {
                        keep = false;
                    }
                }
                if (keep) {
                    float2 sv = {0.f, 0.f};
                    const int b = c.b0 + j;
                    if (ku < c.K && b < c.nrhs) sv = c.S[(int64_t)b * c.lds + d.perm[ku]];
                    float2 q = c.L.Q[ku * 16 + j];
                    c.L.R[ku * 16 + j] = float2{sv.x - sr - c.xi * q.x, sv.y - si - c.xi * q.y};
                }
            }
        }
        __syncthreads();
    }
}

// phi <- r / ||a||^2 on the rows with sel (0 elsewhere) of the active
// columns, in place over R; per-column num = sum |r|^2/||a||^2 and ||phi||^2.
// sel: 0 all rows, 1 rows of F, 2 rows of V.
template <int W>
__device__ __forceinline__ void tile_phi(const TileCtx &c, int sel)
{
    const int tid = threadIdx.x, j = tid & 15, er = tid >> 4, rows_per_pass = W * 4;
    const VrkDesc &d = *c.d;
    float nm = 0.f, pf = 0.f;
    const bool act = c.L.active[j] != 0;
    for (int ku = er; ku < c.kpad; ku += rows_per_pass) {
        float2 r = c.L.R[ku * 16 + j];
        float2 f = {0.f, 0.f};
        bool in = ku < c.K;
        if (in && sel) in = (d.inf[d.perm[ku]] != 0) == (sel == 1);
        if (act && in) {
            const float inv = 1.f / c.L.nrm[ku];
            f = float2{r.x * inv, r.y * inv};
            nm += (r.x * r.x + r.y * r.y) * inv;
            pf += f.x * f.x + f.y * f.y;
        }
        c.L.R[ku * 16 + j] = f;
    }
    nm = col_sum<W>(nm, c.L.red);
    pf = col_sum<W>(pf, c.L.red);
    if (tid < 16) {
        c.L.num[tid] = nm;
        c.L.phin[tid] = pf;
    }
    __syncthreads();
}

// P = H^H phi on antenna block ab: chunks e of that block's list, two at a
// time so the loads of one pair overlap the MFMAs of the other.
__device__ __forceinline__ void agg_block(const TileCtx &c, int ab, f4 &pr, f4 &pi)
{
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const VrkDesc &d = *c.d;
    C3 acc = c3_zero();
    const int e0 = c.L.agoff[ab], e1 = c.L.agoff[ab + 1];
    int e = e0;
#pragma unroll 1
    for (; e + 1 < e1; e += 2) {
        const int uc0 = d.ag_uc[e], uc1 = d.ag_uc[e + 1];
        float2 h0 = c.HG[(int64_t)e * 64 + lane], h1 = c.HG[(int64_t)(e + 1) * 64 + lane];
        float2 f0 = c.L.R[(4 * uc0 + g) * 16 + j], f1 = c.L.R[(4 * uc1 + g) * 16 + j];
        c3mfma(acc, h0, f0);
        c3mfma(acc, h1, f1);
    }
    if (e < e1) {
        const int uc = d.ag_uc[e];
        c3mfma(acc, c.HG[(int64_t)e * 64 + lane], c.L.R[(4 * uc + g) * 16 + j]);
    }
    c3_get(acc, pr, pi);
}

// Aggregated projection (update4): x += gamma H^H phi, q += gamma phi with
// gamma = phi^H r / ||A^H phi||^2. The denominator is evaluated through the
// Gram identity ||A^H phi||^2 = ||H^H phi||^2 + xi ||phi||^2
// = phi^H (H H^H + xi I) phi on the Gram tiles, so gamma is known before
// P = H^H phi is formed and P goes straight into x (one pass).
template <int W, int NA>
__device__ __forceinline__ void tile_aggregate(const TileCtx &c, f4 (&xr)[NA ? NA : 1], f4 (&xq)[NA ? NA : 1])
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, j = lane & 15, g = lane >> 4;
    const int er = tid >> 4, rows_per_pass = W * 4;
    const VrkDesc &d = *c.d;
    // phi^H M phi: row blocks mb of M phi on the waves, dotted with phi
    float den = 0.f;
#pragma unroll 1
    for (int mb = w; mb < c.nub; mb += W) {
        C3 acc = c3_zero();
        const int e0 = c.L.gmoff[mb], e1 = c.L.gmoff[mb + 1];
#pragma unroll 1
        for (int e = e0; e < e1; ++e) {
            const int uc = d.gm_c[e];
            c3mfma(acc, c.GM[(int64_t)e * 64 + lane], c.L.R[(4 * uc + g) * 16 + j]);
        }
        f4 mr, mi;
        c3_get(acc, mr, mi);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float2 f = c.L.R[(16 * mb + 4 * g + r) * 16 + j];
            den += f.x * mr[r] + f.y * mi[r];
        }
    }
    den = col_sum<W>(den, c.L.red);
    if (tid < 16) {
        const float num = c.L.num[tid];
        c.L.gre[tid] = (c.L.active[tid] && num > 0.f && den > 0.f) ? num / den : 0.f;
    }
    __syncthreads();
    const float gm = c.L.gre[j];
    if constexpr (NA == 0) {
#pragma unroll 1
        for (int ab = w; ab < c.nab; ab += W) {
            f4 qr, qi;
            agg_block(c, ab, qr, qi);
            float2 *xp = c.Xw + (int64_t)ab * 256 + lane;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float2 x = xp[64 * r];
                xp[64 * r] = float2{x.x + gm * qr[r], x.y + gm * qi[r]};
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const int ab = w + W * t;
            if (ab < c.nab) {
                f4 qr, qi;
                agg_block(c, ab, qr, qi);
                xr[t] += gm * qr;
                xq[t] += gm * qi;
            }
        }
    }
    for (int ku = er; ku < c.kpad; ku += rows_per_pass) {
        float2 f = c.L.R[ku * 16 + j];
        float2 q = c.L.Q[ku * 16 + j];
        c.L.Q[ku * 16 + j] = float2{q.x + gm * f.x, q.y + gm * f.y};
    }
    __syncthreads();
}

template <int W, int NA, int VARIANT>
__device__ __forceinline__ void solve_item(const VrkSolveArgs &a, const VrkWork wk, char *smem)
{
    const VrkDesc &d = a.desc[wk.prob];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, j = lane & 15, g = lane >> 4;
    TileCtx c;
    c.d = &d;
    c.prob = wk.prob;
    c.K = d.k;
    c.N = d.nt;
    c.nub = d.nub;
    c.kpad = d.nub * VRK_UB;
    c.nab = d.nab;
    c.xi = (float)d.xi;
    c.b0 = wk.tile * VRK_TILE_RHS;
    c.nrhs = d.nrhs;
    mfma_lds_layout(c.kpad, c.nab, W, smem, &c.L);
    const MfmaLds &L = c.L;
    float2 *X, *V;
    int64_t ldx_, ldv_;
    if (a.adjoint) {
        c.S = reinterpret_cast<const float2 *>(d.Sadj); c.lds = c.K;
        X = reinterpret_cast<float2 *>(d.Xadj); ldx_ = c.N;
        V = reinterpret_cast<float2 *>(d.GS); ldv_ = d.ldgs;
    } else {
        c.S = reinterpret_cast<const float2 *>(d.S); c.lds = d.lds;
        X = reinterpret_cast<float2 *>(d.X); ldx_ = d.ldx;
        V = reinterpret_cast<float2 *>(d.V); ldv_ = d.ldv;
    }
    c.H = reinterpret_cast<const float2 *>(d.H);
    c.HA = reinterpret_cast<const float2 *>(d.HA);
    c.HG = reinterpret_cast<const float2 *>(d.HG);
    c.GM = reinterpret_cast<const float2 *>(d.GM);
    c.Xw = NA == 0 ? reinterpret_cast<float2 *>(d.Xw) + (int64_t)wk.tile * c.nab * 256 : nullptr;
    const float *nrm_g = reinterpret_cast<const float *>(d.nrm);
    const int K = c.K, N = c.N, kpad = c.kpad, b0 = c.b0;
    const int rows_per_pass = W * 4;   // (row, column) entries: tid -> (tid / 16, tid % 16)
    const int er = tid >> 4;

    // ---- init: x = 0, q = 0, r = s (z0 = 0), norms in VR-start order
    constexpr int NR = NA ? NA : 1;
    f4 xr[NR], xq[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        xr[t] = f4{0.f, 0.f, 0.f, 0.f};
        xq[t] = f4{0.f, 0.f, 0.f, 0.f};
    }
    if constexpr (NA == 0)
        for (int ab = w; ab < c.nab; ab += W)
#pragma unroll
            for (int r = 0; r < 4; ++r) c.Xw[(int64_t)ab * 256 + 64 * r + lane] = float2{0.f, 0.f};
    float s2 = 0.f;
    for (int ku = er; ku < kpad; ku += rows_per_pass) {
        float2 sv = {0.f, 0.f};
        const int b = b0 + j;
        if (ku < K && b < c.nrhs) sv = c.S[(int64_t)b * c.lds + d.perm[ku]];
        L.R[ku * 16 + j] = sv;
        L.Q[ku * 16 + j] = float2{0.f, 0.f};
        s2 += sv.x * sv.x + sv.y * sv.y;
    }
    for (int ku = tid; ku < kpad; ku += W * 64) {
        L.nrm[ku] = ku < K ? nrm_g[d.perm[ku]] : 1.f;
        if (ku < K) L.posl[d.perm[ku]] = ku;
    }
    for (int i = tid; i <= c.nab; i += W * 64) L.agoff[i] = d.ag_off[i];
    for (int i = tid; i <= c.nub; i += W * 64) L.gmoff[i] = d.gm_off[i];
    for (int i = tid; i < c.nub; i += W * 64) {
        L.rlo[i] = d.rab_lo[i];
        L.rhi[i] = d.rab_hi[i];
        L.hoff[i] = (int)d.ha_off[i];
    }
    s2 = col_sum<W>(s2, L.red);
    const float fro2 = *reinterpret_cast<const float *>(d.fro2);
    if (tid < 16) {
        const int b = b0 + tid;
        float sn = sqrtf(s2);
        L.snorm[tid] = sn;
        int act = 0, fl = 0;
        if (b < c.nrhs) {
            if (!isfinite(sn) || !isfinite(fro2)) fl = VRK_FLAG_NONFINITE;
            else if (s2 == 0.f) fl = VRK_FLAG_CONVERGED;
            else act = 1;
        }
        L.active[tid] = act;
        L.flags[tid] = fl;
        L.iters[tid] = 0;
        L.rel[tid] = 0.f;
        L.pick[tid] = -1;
    }
    __syncthreads();

    constexpr int variant = VARIANT;
    int64_t t_it = 0;
    for (;;) {
        if (t_it > 0) tile_residual<W, NA>(c, xr, xq, variant == 2);
        // stop rule per column
        float r2 = 0.f;
        for (int ku = er; ku < kpad; ku += rows_per_pass) {
            float2 r = L.R[ku * 16 + j];
            r2 += r.x * r.x + r.y * r.y;
        }
        r2 = col_sum<W>(r2, L.red);
        if (tid < 16) {
            if (L.active[tid]) {
                const float rel = sqrtf(r2) / L.snorm[tid];
                L.rel[tid] = rel;
                L.iters[tid] = (int)t_it;
                if (!isfinite(rel)) { L.flags[tid] = VRK_FLAG_NONFINITE; L.active[tid] = 0; }
                else if (rel <= (float)a.tol) { L.flags[tid] = VRK_FLAG_CONVERGED; L.active[tid] = 0; }
                else if (t_it >= a.max_iters) { L.flags[tid] = VRK_FLAG_MAXITER; L.active[tid] = 0; }
            }
        }
        __syncthreads();
        if (tid == 0) {
            int any = 0;
            for (int cc = 0; cc < 16; ++cc) any |= L.active[cc];
            *L.any = any;
        }
        __syncthreads();
        if (!*L.any) break;

        if constexpr (variant == 0 || variant == 2) {
            // greedy selection, one wave per column
            for (int cc = w; cc < 16; cc += W) {
                if (!L.active[cc]) {
                    if (lane == 0) { L.gre[cc] = 0.f; L.gim[cc] = 0.f; }
                    continue;
                }
                const float u = (float)uniform24(a.seed, t_it, b0 + cc, c.prob);
                const float2 *Rl = L.R;
                const float *nl = L.nrm;
                const int *pl = L.posl;
                const int i = select_row_wave<float>(K, a.select, fro2, u, [Rl, nl, pl, cc](int q) -> cx<float> {
                    const int ku = pl[q];
                    float2 r = Rl[ku * 16 + cc];
                    return {r.x * r.x + r.y * r.y, nl[ku]};
                }, L.pre + w * kpad);
                if (lane == 0) {
                    const int ku = L.posl[i];
                    const float inv = 1.f / L.nrm[ku];
                    float2 r = L.R[ku * 16 + cc];
                    L.pick[cc] = i;
                    L.gre[cc] = r.x * inv;
                    L.gim[cc] = r.y * inv;
                }
            }
            __syncthreads();
            // single-row projection per column: x += gamma conj(H[i, VR_i])
            {
                const int i = L.pick[j];
                const float gr = L.gre[j], gi = L.gim[j];
                if (NA == 0 && i >= 0 && (gr != 0.f || gi != 0.f)) {
                    const int s0 = d.vs[i], e0 = d.ve[i];
                    const float2 *hrow = c.H + (int64_t)i * d.ldh;
                    for (int ab = w; ab < c.nab; ab += W) {
                        const int nb = 16 * ab + 4 * g;
                        if (nb + 3 < s0 || nb >= e0) continue;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int n = nb + r;
                            if (n >= s0 && n < e0) {
                                float2 h = hrow[n];
                                float2 *xp = c.Xw + (int64_t)ab * 256 + 64 * r + lane;
                                float2 x = *xp;
                                *xp = float2{x.x + gr * h.x + gi * h.y, x.y + gi * h.x - gr * h.y};
                            }
                        }
                    }
                }
                if (NA > 0 && i >= 0 && (gr != 0.f || gi != 0.f)) {
                    const int s0 = d.vs[i], e0 = d.ve[i];
                    const float2 *hrow = c.H + (int64_t)i * d.ldh;
#pragma unroll
                    for (int t = 0; t < NA; ++t) {
                        const int nb = 16 * (w + W * t) + 4 * g;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int n = nb + r;
                            if (n >= s0 && n < e0) {
                                float2 h = hrow[n];
                                xr[t][r] += gr * h.x + gi * h.y;
                                xq[t][r] += gi * h.x - gr * h.y;
                            }
                        }
                    }
                }
            }
            if (tid < 16 && L.active[tid]) {
                const int ku = L.posl[L.pick[tid]];
                float2 q = L.Q[ku * 16 + tid];
                L.Q[ku * 16 + tid] = float2{q.x + L.gre[tid], q.y + L.gim[tid]};
            }
            __syncthreads();
        } else if constexpr (variant == 1) {
            tile_phi<W>(c, 0);
            tile_aggregate<W, NA>(c, xr, xq);
        } else {
            // orthogonal half-step on F with gamma = 1 (Prop. 1); each antenna
            // belongs to at most one user of F
            tile_phi<W>(c, 1);
            if constexpr (NA == 0) {
                for (int ab = w; ab < c.nab; ab += W) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int n = 16 * ab + 4 * g + r;
                        if (n < N) {
                            const int o = d.fown[n];
                            if (o >= 0) {
                                float2 f = L.R[o * 16 + j];
                                float2 h = c.H[(int64_t)d.perm[o] * d.ldh + n];
                                float2 *xp = c.Xw + (int64_t)ab * 256 + 64 * r + lane;
                                float2 x = *xp;
                                *xp = float2{x.x + f.x * h.x + f.y * h.y, x.y + f.y * h.x - f.x * h.y};
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                const int nb = 16 * (w + W * t) + 4 * g;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = nb + r;
                    if (n < N) {
                        const int o = d.fown[n];
                        if (o >= 0) {
                            float2 f = L.R[o * 16 + j];
                            float2 h = c.H[(int64_t)d.perm[o] * d.ldh + n];
                            xr[t][r] += f.x * h.x + f.y * h.y;
                            xq[t][r] += f.y * h.x - f.x * h.y;
                        }
                    }
                }
            }
            for (int ku = er; ku < kpad; ku += rows_per_pass) {
                float2 f = L.R[ku * 16 + j];
                float2 q = L.Q[ku * 16 + j];
                L.Q[ku * 16 + j] = float2{q.x + f.x, q.y + f.y};
            }
            __syncthreads();
            if (d.nv > 0) {
                tile_residual<W, NA>(c, xr, xq, false);
                tile_phi<W>(c, 2);
                tile_aggregate<W, NA>(c, xr, xq);
            }
        }
        ++t_it;
    }

    // ---- outputs
    {
        const int b = b0 + j;
        if (b < c.nrhs) {
            if constexpr (NA == 0)
                for (int ab = w; ab < c.nab; ab += W)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int n = 16 * ab + 4 * g + r;
                        if (n < N) X[(int64_t)b * ldx_ + n] = c.Xw[(int64_t)ab * 256 + 64 * r + lane];
                    }
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                const int nb = 16 * (w + W * t) + 4 * g;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = nb + r;
                    if (n < N) X[(int64_t)b * ldx_ + n] = float2{xr[t][r], xq[t][r]};
                }
            }
            if (V)
                for (int ku = er; ku < K; ku += rows_per_pass)
                    V[(int64_t)b * ldv_ + d.perm[ku]] = L.Q[ku * 16 + j];
        }
    }
    if (tid < 16) {
        const int b = b0 + tid;
        if (b < c.nrhs) {
            const int64_t gidx = d.rhs_base + b;
            if (a.iters) a.iters[gidx] = L.iters[tid];
            if (a.relres) a.relres[gidx] = L.rel[tid];
            if (a.flags) a.flags[gidx] = L.flags[tid];
        }
    }
}


// Next work item of this workgroup: its own XCD's queue first, then the
// others in turn; -1 when every queue is drained. Queue q holds the work
// items [qbase[q], qbase[q] + qsize[q]) and its counter qcount[q].
__device__ __forceinline__ int next_item(const VrkQueue &q, int *sh)
{
    if (threadIdx.x == 0) {
        const int x = blockIdx.x % VRK_NQUEUE;
        int item = -1;
        for (int s = 0; s < VRK_NQUEUE && item < 0; ++s) {
            const int qi = (x + s) % VRK_NQUEUE;
            const int pos = atomicAdd(q.count + qi, 1);
            if (pos < q.size[qi]) item = q.base[qi] + pos;
        }
        *sh = item;
    }
    __syncthreads();
    const int item = *sh;
    __syncthreads();
    return item;
}

template <int W, int NA, int VARIANT, bool PERSIST>
__global__ void __launch_bounds__(W * 64) k_mfma_solve(VrkSolveArgs a, const VrkWork *work, VrkQueue q)
{
    extern __shared__ __align__(16) char smem[];
    if constexpr (!PERSIST) {
        solve_item<W, NA, VARIANT>(a, work[blockIdx.x], smem);   // one workgroup per work item
    } else {
        __shared__ int sh_item;
        for (int item = next_item(q, &sh_item); item >= 0; item = next_item(q, &sh_item))
            solve_item<W, NA, VARIANT>(a, work[item], smem);
    }
}

__global__ void k_queue_reset(int *count)
{
    if (threadIdx.x < VRK_NQUEUE) count[threadIdx.x] = 0;
}

// Launch (mode 0), set the LDS attribute and report occupancy (mode 1).
template <int W, int NA, int VARIANT, bool PERSIST>
hipError_t launch_kernel(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid,
                         size_t lds, hipStream_t s, int mode, int *blocks_per_cu)
{
    auto kern = k_mfma_solve<W, NA, VARIANT, PERSIST>;
    if (mode == 1) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, W * 64, lds);
    }
    if (PERSIST) hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, q.count);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(W * 64), lds, s, a, work, q);
    return hipGetLastError();
}

template <int W, int NA, int VARIANT>
hipError_t launch_one(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid, size_t lds,
                      hipStream_t s, int mode, int *blocks_per_cu)
{
    if (q.count) return launch_kernel<W, NA, VARIANT, true>(a, work, q, grid, lds, s, mode, blocks_per_cu);
    return launch_kernel<W, NA, VARIANT, false>(a, work, q, grid, lds, s, mode, blocks_per_cu);
}

template <int W, int NA>
hipError_t launch_variant(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid, size_t lds,
                          hipStream_t s, int mode, int *bpc)
{
    switch (a.variant) {
    case 0: return launch_one<W, NA, 0>(a, work, q, grid, lds, s, mode, bpc);
    case 1: return launch_one<W, NA, 1>(a, work, q, grid, lds, s, mode, bpc);
    case 2: return launch_one<W, NA, 2>(a, work, q, grid, lds, s, mode, bpc);
    case 3: return launch_one<W, NA, 3>(a, work, q, grid, lds, s, mode, bpc);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// x of one tile lives in registers when it fits: at most 16 antenna blocks
// per wave with 8 waves (two waves per SIMD) and 8 with 16 waves (four per
// SIMD), i.e. Nt <= 2048. Larger Nt keeps x in a workspace buffer (NA = 0).
int vrk_mfma_supported(int32_t nt, int32_t waves)
{
    (void)nt;
    return waves == 8 || waves == 16;
}

int vrk_mfma_register_na(int32_t nt, int32_t waves)
{
    const int nab = (nt + VRK_AB - 1) / VRK_AB;
    const int cap = waves == 8 ? 16 : 8;
    int na = (nab + waves - 1) / waves, nap = 1;
    while (nap < na) nap *= 2;
    return nap <= cap ? nap : 0;
}

size_t vrk_mfma_lds_bytes(int32_t kpad, int32_t nab, int32_t waves)
{
    return mfma_lds_layout(kpad, nab, waves, nullptr, nullptr);
}

hipError_t vrk_launch_mfma_solve(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid,
                                 int32_t waves, int32_t na, size_t lds, hipStream_t s, int mode, int *bpc)
{
    if (grid <= 0) return hipSuccess;
#define VRK_NA_CASES(W)                                                          \
    switch (na) {                                                                \
    case 1: return launch_variant<W, 1>(a, work, q, grid, lds, s, mode, bpc);    \
    case 2: return launch_variant<W, 2>(a, work, q, grid, lds, s, mode, bpc);    \
    case 4: return launch_variant<W, 4>(a, work, q, grid, lds, s, mode, bpc);    \
    case 8: return launch_variant<W, 8>(a, work, q, grid, lds, s, mode, bpc);    \
    }
    if (waves == 8) {
        if (na == 16) return launch_variant<8, 16>(a, work, q, grid, lds, s, mode, bpc);
        if (na == 0) return launch_variant<8, 0>(a, work, q, grid, lds, s, mode, bpc);
        VRK_NA_CASES(8)
    } else if (waves == 16) {
        if (na == 0) return launch_variant<16, 0>(a, work, q, grid, lds, s, mode, bpc);
        VRK_NA_CASES(16)
    }
#undef VRK_NA_CASES
    return hipErrorInvalidValue;
}
