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
    float *nrm, *pre, *red, *snorm, *rel, *gre, *gim;
    int *posl, *active, *iters, *flags, *pick;
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
    char *red = take((size_t)2 * W * 16 * 4);
    char *sc = take(16 * 4 * 4);
    char *posl = take((size_t)kpad * 4);
    char *ints = take(16 * 4 * 4);
    char *tabs = take((size_t)(nab + 1 + 4 * (kpad / 16) + 1) * 4);
    // test the LDS base, not L: L points into a caller's register-resident
    // struct, and comparing its address would pin that struct to memory
    if (base) {
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
        L->posl = (int *)posl;
        int *ip = (int *)ints;
        L->active = ip;
        L->iters = ip + 16;
        L->flags = ip + 32;
        L->pick = ip + 48;
    }
    return off;
}

// Sums over the threads of each RHS column j = tid % 16; every thread gets
// its column's totals. Two barriers: one before the per-wave partials are
// written (earlier readers of the buffer are done), one after. Fixed order.
template <int W>
__device__ __forceinline__ float col_sum(float v, float *red)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    __syncthreads();
    if (lane < 16) red[w * 16 + lane] = v;
    __syncthreads();
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < W; ++i) s += red[i * 16 + (tid & 15)];
    return s;
}

template <int W>
__device__ __forceinline__ float2 col_sum2(float a, float b, float *red)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    a += __shfl_xor(a, 16, 64);
    a += __shfl_xor(a, 32, 64);
    b += __shfl_xor(b, 16, 64);
    b += __shfl_xor(b, 32, 64);
    __syncthreads();
    if (lane < 16) {
        red[w * 16 + lane] = a;
        red[(W + w) * 16 + lane] = b;
    }
    __syncthreads();
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        sa += red[i * 16 + (tid & 15)];
        sb += red[(W + i) * 16 + (tid & 15)];
    }
    return float2{sa, sb};
}

// Per-tile constants shared by the phases below (passed by value so that
// everything stays in registers after inlining).
using CDesc = const VRK_CONST VrkDesc;
template <typename T>
using gp = VRK_GLOBAL T *;

struct TileCtx {
    MfmaLds L;
    gp<const float2> S, H, HA, HG, GM, FH;
    gp<float2> Xw;   // global-iterate mode: this tile's x, [ab][r][lane] (MFMA result order)
    gp<const int32_t> perm, vs, ve, ag_uc, gm_c, fown;
    gp<const uint8_t> inf;
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
                        const gp<const float2> hp = c.HA + (hb + 4 * (int64_t)(ab - lo)) * 64 + lane;
                        const gp<const float2> xp = c.Xw + (int64_t)ab * 256 + lane;
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
                            const gp<const float2> hp = c.HA + (hb + 4 * (int64_t)(ab - lo)) * 64 + lane;
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
                        const int u = c.perm[ku];
                        keep = (u == pk) || (max(c.vs[u], c.vs[pk]) < min(c.ve[u], c.ve[pk]));
                    } else {
                        keep = false;
                    }
                }
                if (keep) {
                    float2 sv = {0.f, 0.f};
                    const int b = c.b0 + j;
                    if (ku < c.K && b < c.nrhs) sv = c.S[(int64_t)b * c.lds + c.perm[ku]];
                    float2 q = c.L.Q[ku * 16 + j];
                    c.L.R[ku * 16 + j] = float2{sv.x - sr - c.xi * q.x, sv.y - si - c.xi * q.y};
                }
            }
        }
        __syncthreads();
    }
}

// phi <- r / ||a||^2 on the rows with sel (0 elsewhere) of the active
// columns, in place over R. Returns, for the calling thread's column,
// num = sum |r_i|^2/||a_i||^2 over the rows and ||phi||^2.
// sel: 0 all rows, 1 rows of F, 2 rows of V.
template <int W>
__device__ __forceinline__ float2 tile_phi(const TileCtx &c, int sel)
{
    const int tid = threadIdx.x, j = tid & 15, er = tid >> 4, rows_per_pass = W * 4;
    float nm = 0.f, pf = 0.f;
    const bool act = c.L.active[j] != 0;
    for (int ku = er; ku < c.kpad; ku += rows_per_pass) {
        float2 r = c.L.R[ku * 16 + j];
        float2 f = {0.f, 0.f};
        bool in = ku < c.K;
        if (in && sel) in = (c.inf[c.perm[ku]] != 0) == (sel == 1);
        if (act && in) {
            const float inv = 1.f / c.L.nrm[ku];
            f = float2{r.x * inv, r.y * inv};
            nm += (r.x * r.x + r.y * r.y) * inv;
            pf += f.x * f.x + f.y * f.y;
        }
        c.L.R[ku * 16 + j] = f;
    }
    return col_sum2<W>(nm, pf, c.L.red);
}

// P = H^H phi on antenna block ab: chunks e of that block's list, two at a
// time so the loads of one pair overlap the MFMAs of the other.
__device__ __forceinline__ void agg_block(const TileCtx &c, int ab, f4 &pr, f4 &pi)
{
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    C3 acc = c3_zero();
    const int e0 = c.L.agoff[ab], e1 = c.L.agoff[ab + 1];
    int e = e0;
#pragma unroll 1
    for (; e + 1 < e1; e += 2) {
        const int uc0 = c.ag_uc[e], uc1 = c.ag_uc[e + 1];
        float2 h0 = c.HG[(int64_t)e * 64 + lane], h1 = c.HG[(int64_t)(e + 1) * 64 + lane];
        float2 f0 = c.L.R[(4 * uc0 + g) * 16 + j], f1 = c.L.R[(4 * uc1 + g) * 16 + j];
        c3mfma(acc, h0, f0);
        c3mfma(acc, h1, f1);
    }
    if (e < e1) {
        const int uc = c.ag_uc[e];
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
__device__ __forceinline__ void tile_aggregate(const TileCtx &c, f4 (&xr)[NA ? NA : 1], f4 (&xq)[NA ? NA : 1],
                                               float num)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, j = lane & 15, g = lane >> 4;
    const int er = tid >> 4, rows_per_pass = W * 4;
    // phi^H M phi: row blocks mb of M phi on the waves, dotted with phi
    float den = 0.f;
#pragma unroll 1
    for (int mb = w; mb < c.nub; mb += W) {
        C3 acc = c3_zero();
        const int e0 = c.L.gmoff[mb], e1 = c.L.gmoff[mb + 1];
#pragma unroll 1
        for (int e = e0; e < e1; ++e) {
            const int uc = c.gm_c[e];
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
    const float gm = (c.L.active[j] && num > 0.f && den > 0.f) ? num / den : 0.f;
    if constexpr (NA == 0) {
#pragma unroll 1
        for (int ab = w; ab < c.nab; ab += W) {
            f4 qr, qi;
            agg_block(c, ab, qr, qi);
            const gp<float2> xp = c.Xw + (int64_t)ab * 256 + lane;
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
    // each thread updates its own (row, column) entries; the next phase reads
    // Q and rewrites R only after a barrier of its own
    for (int ku = er; ku < c.kpad; ku += rows_per_pass) {
        float2 f = c.L.R[ku * 16 + j];
        float2 q = c.L.Q[ku * 16 + j];
        c.L.Q[ku * 16 + j] = float2{q.x + gm * f.x, q.y + gm * f.y};
    }
    if constexpr (NA == 0) __syncthreads();   // the residual reads every wave's x blocks
}

template <int W, int NA, int VARIANT>
__device__ __forceinline__ void solve_item(const VrkSolveArgs &a, const int prob, const int tile, char *smem)
{
    // prob and tile are wave-uniform, so the descriptor is read with scalar loads
    CDesc &d = ((CDesc *)a.desc)[prob];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, j = lane & 15, g = lane >> 4;
    TileCtx c;
    c.prob = prob;
    c.K = d.k;
    c.N = d.nt;
    c.nub = d.nub;
    c.kpad = d.nub * VRK_UB;
    c.nab = d.nab;
    c.xi = (float)d.xi;
    c.b0 = tile * VRK_TILE_RHS;
    c.nrhs = d.nrhs;
    mfma_lds_layout(c.kpad, c.nab, W, smem, &c.L);
    const MfmaLds &L = c.L;
    gp<float2> X, V;
    int64_t ldx_, ldv_;
    if (a.adjoint) {
        c.S = gmem(static_cast<const float2 *>(d.Sadj)); c.lds = c.K;
        X = gmem(static_cast<float2 *>(d.Xadj)); ldx_ = c.N;
        V = gmem(static_cast<float2 *>(d.GS)); ldv_ = d.ldgs;
    } else {
        c.S = gmem(static_cast<const float2 *>(d.S)); c.lds = d.lds;
        X = gmem(static_cast<float2 *>(d.X)); ldx_ = d.ldx;
        V = gmem(static_cast<float2 *>(d.V)); ldv_ = d.ldv;
    }
    c.H = gmem(static_cast<const float2 *>(d.H));
    c.HA = gmem(static_cast<const float2 *>(d.HA));
    c.HG = gmem(static_cast<const float2 *>(d.HG));
    c.GM = gmem(static_cast<const float2 *>(d.GM));
    c.FH = gmem(static_cast<const float2 *>(d.FH));
    c.Xw = NA == 0 ? gmem(static_cast<float2 *>(d.Xw)) + (int64_t)tile * c.nab * 256 : nullptr;
    c.perm = gmem(d.perm);
    c.vs = gmem(d.vs);
    c.ve = gmem(d.ve);
    c.ag_uc = gmem(d.ag_uc);
    c.gm_c = gmem(d.gm_c);
    c.fown = gmem(d.fown);
    c.inf = gmem(d.inf);
    const gp<const float> nrm_g = gmem(static_cast<const float *>(d.nrm));
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
        if (ku < K && b < c.nrhs) sv = c.S[(int64_t)b * c.lds + c.perm[ku]];
        L.R[ku * 16 + j] = sv;
        L.Q[ku * 16 + j] = float2{0.f, 0.f};
        s2 += sv.x * sv.x + sv.y * sv.y;
    }
    for (int ku = tid; ku < kpad; ku += W * 64) {
        L.nrm[ku] = ku < K ? nrm_g[c.perm[ku]] : 1.f;
        if (ku < K) L.posl[c.perm[ku]] = ku;
    }
    for (int i = tid; i <= c.nab; i += W * 64) L.agoff[i] = gmem(d.ag_off)[i];
    for (int i = tid; i <= c.nub; i += W * 64) L.gmoff[i] = gmem(d.gm_off)[i];
    for (int i = tid; i < c.nub; i += W * 64) {
        L.rlo[i] = gmem(d.rab_lo)[i];
        L.rhi[i] = gmem(d.rab_hi)[i];
        L.hoff[i] = (int)gmem(d.ha_off)[i];
    }
    s2 = col_sum<W>(s2, L.red);
    const float fro2 = *gmem(static_cast<const float *>(d.fro2));
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
        // every lane evaluates its column's stop rule; lanes 0..15 of each wave
        // cover all 16 columns, so a ballot tells whether any stays active
        bool still = false;
        {
            const bool was = L.active[j] != 0;
            const float rel = sqrtf(r2) / L.snorm[j];
            int fl = 0;
            if (was) {
                if (!isfinite(rel)) fl = VRK_FLAG_NONFINITE;
                else if (rel <= (float)a.tol) fl = VRK_FLAG_CONVERGED;
                else if (t_it >= a.max_iters) fl = VRK_FLAG_MAXITER;
                still = fl == 0;
            }
            __syncthreads();   // every lane has read its column's old state
            if (tid < 16 && was) {
                L.rel[tid] = rel;
                L.iters[tid] = (int)t_it;
                if (fl) {
                    L.flags[tid] = fl;
                    L.active[tid] = 0;
                }
            }
        }
        const bool any = __ballot(still) != 0;
        __syncthreads();
        if (!any) break;

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
                    const int s0 = c.vs[i], e0 = c.ve[i];
                    const gp<const float2> hrow = c.H + (int64_t)i * d.ldh;
                    for (int ab = w; ab < c.nab; ab += W) {
                        const int nb = 16 * ab + 4 * g;
                        if (nb + 3 < s0 || nb >= e0) continue;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int n = nb + r;
                            if (n >= s0 && n < e0) {
                                float2 h = hrow[n];
                                const gp<float2> xp = c.Xw + (int64_t)ab * 256 + 64 * r + lane;
                                float2 x = *xp;
                                *xp = float2{x.x + gr * h.x + gi * h.y, x.y + gi * h.x - gr * h.y};
                            }
                        }
                    }
                }
                if (NA > 0 && i >= 0 && (gr != 0.f || gi != 0.f)) {
                    const int s0 = c.vs[i], e0 = c.ve[i];
                    const gp<const float2> hrow = c.H + (int64_t)i * d.ldh;
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
            const float2 nf = tile_phi<W>(c, 0);
            tile_aggregate<W, NA>(c, xr, xq, nf.x);
        } else {
            // orthogonal half-step on F with gamma = 1 (Prop. 1); each antenna
            // belongs to at most one user of F
            (void)tile_phi<W>(c, 1);
            // x_n += phi_o conj(H[o, n]) for the F owner o of antenna n; a lane
            // reads the owners and H entries of its 4 antennas as vectors
            auto fstep = [&](int nb, float (&xre)[4], float (&xim)[4]) {
                const int4 o4 = *(gp<const int4>)(c.fown + nb);
                const float4 h01 = *(gp<const float4>)(c.FH + nb);
                const float4 h23 = *(gp<const float4>)(c.FH + nb + 2);
                const int o[4] = {o4.x, o4.y, o4.z, o4.w};
                const float hr[4] = {h01.x, h01.z, h23.x, h23.z}, hi[4] = {h01.y, h01.w, h23.y, h23.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float2 f = o[r] >= 0 ? L.R[o[r] * 16 + j] : float2{0.f, 0.f};
                    xre[r] += f.x * hr[r] + f.y * hi[r];
                    xim[r] += f.y * hr[r] - f.x * hi[r];
                }
            };
            if constexpr (NA == 0) {
                for (int ab = w; ab < c.nab; ab += W) {
                    const gp<float2> xp = c.Xw + (int64_t)ab * 256 + lane;
                    float xre[4], xim[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float2 x = xp[64 * r];
                        xre[r] = x.x;
                        xim[r] = x.y;
                    }
                    fstep(16 * ab + 4 * g, xre, xim);
#pragma unroll
                    for (int r = 0; r < 4; ++r) xp[64 * r] = float2{xre[r], xim[r]};
                }
            }
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                const int ab = w + W * t;
                if (ab < c.nab) {
                    float xre[4] = {xr[t][0], xr[t][1], xr[t][2], xr[t][3]};
                    float xim[4] = {xq[t][0], xq[t][1], xq[t][2], xq[t][3]};
                    fstep(16 * ab + 4 * g, xre, xim);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        xr[t][r] = xre[r];
                        xq[t][r] = xim[r];
                    }
                }
            }
            for (int ku = er; ku < kpad; ku += rows_per_pass) {
                float2 f = L.R[ku * 16 + j];
                float2 q = L.Q[ku * 16 + j];
                L.Q[ku * 16 + j] = float2{q.x + f.x, q.y + f.y};
            }
            if constexpr (NA == 0) __syncthreads();   // the residual reads every wave's x blocks
            if (d.nv > 0) {
                tile_residual<W, NA>(c, xr, xq, false);
                const float2 nf = tile_phi<W>(c, 2);
                tile_aggregate<W, NA>(c, xr, xq, nf.x);
            }
        }
        ++t_it;
    }

    // ---- outputs. Each lane holds 4 consecutive antennas of one RHS: two
    // 16-byte stores when the row is 32-byte aligned, else four 8-byte ones.
    {
        const int b = b0 + j;
        if (b < c.nrhs) {
            const gp<float2> xrow = X + (int64_t)b * ldx_;
            const bool vec = ((reinterpret_cast<uintptr_t>(xrow) & 31) == 0);
            auto put4 = [&](int nb, float2 v0, float2 v1, float2 v2, float2 v3) {
                if (vec && nb + 3 < N) {
                    const gp<float4> p4 = (gp<float4>)(xrow + nb);
                    p4[0] = float4{v0.x, v0.y, v1.x, v1.y};
                    p4[1] = float4{v2.x, v2.y, v3.x, v3.y};
                } else {
                    if (nb < N) xrow[nb] = v0;
                    if (nb + 1 < N) xrow[nb + 1] = v1;
                    if (nb + 2 < N) xrow[nb + 2] = v2;
                    if (nb + 3 < N) xrow[nb + 3] = v3;
                }
            };
            if constexpr (NA == 0)
                for (int ab = w; ab < c.nab; ab += W) {
                    const gp<const float2> xp = c.Xw + (int64_t)ab * 256 + lane;
                    put4(16 * ab + 4 * g, xp[0], xp[64], xp[128], xp[192]);
                }
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                const int nb = 16 * (w + W * t) + 4 * g;
                put4(nb, float2{xr[t][0], xq[t][0]}, float2{xr[t][1], xq[t][1]}, float2{xr[t][2], xq[t][2]},
                     float2{xr[t][3], xq[t][3]});
            }
            if (V)
                for (int ku = er; ku < K; ku += rows_per_pass)
                    V[(int64_t)b * ldv_ + c.perm[ku]] = L.Q[ku * 16 + j];
        }
    }
    if (tid < 16) {
        const int b = b0 + tid;
        if (b < c.nrhs) {
            const int64_t gidx = d.rhs_base + b;
            if (a.iters) gmem(a.iters)[gidx] = L.iters[tid];
            if (a.relres) gmem(a.relres)[gidx] = L.rel[tid];
            if (a.flags) gmem(a.flags)[gidx] = L.flags[tid];
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
    const int item = __builtin_amdgcn_readfirstlane(*sh);
    __syncthreads();
    return item;
}

template <int W, int NA, int VARIANT, bool PERSIST>
__global__ void __launch_bounds__(W * 64) k_mfma_solve(VrkSolveArgs a, const VrkWork *work, VrkQueue q)
{
    extern __shared__ __align__(16) char smem[];
    if constexpr (!PERSIST) {
        const VrkWork wk = gmem(work)[blockIdx.x];   // one workgroup per work item
        solve_item<W, NA, VARIANT>(a, __builtin_amdgcn_readfirstlane(wk.prob),
                                   __builtin_amdgcn_readfirstlane(wk.tile), smem);
    } else {
        __shared__ int sh_item;
        for (int item = next_item(q, &sh_item); item >= 0; item = next_item(q, &sh_item)) {
            const VrkWork wk = gmem(work)[item];
            solve_item<W, NA, VARIANT>(a, __builtin_amdgcn_readfirstlane(wk.prob),
                                       __builtin_amdgcn_readfirstlane(wk.tile), smem);
        }
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
