// MFMA engine: 16 right-hand sides per workgroup share H; the complex
// products of every Kaczmarz variant run on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32, complex product as three real products).
//
// Dual-space iteration. Every Kaczmarz step on A z = s, A = [H, sqrt(xi) I],
// adds gamma a_i to z and gamma to q_i, so from z = 0 the iterate always is
// x = H^H q and the residual is r = s - A A^H q = s - M q with the Gram matrix
// M = H H^H + xi I (band-sparse: M[i][k] = 0 unless the VRs of i and k
// overlap, which is the orthogonality of Lemma 1 and Theorem 2). The engine
// therefore keeps r and q (K x 16 per tile) in LDS and updates r with Gram
// products, r -= M (gamma phi): the same iterates as the paper's updates of
// x and the re-evaluated residuals, at the cost of the Gram band instead of
// the channel band per step. When every column has met the stop rule, x =
// H^H q is formed and the residual s - M q is evaluated afresh from q (equal
// to s - H x - xi q in exact arithmetic, free of the maintained residual's
// drift); a column whose fresh residual misses the tolerance resumes from it.
//
// Layout. Lane l of a wave is (j, g) = (l % 16, l / 16): RHS column j and
// row group g. Thread (er, j) of the workgroup keeps the entries (er + 4 W k,
// j), k < EP, of r, q and phi in registers; LDS holds phi as the operand of
// the Gram products, their per-wave partials and, for the greedy selection,
// r. x = H^H q is formed once, straight into the output rows: the MFMA
// result tile of antenna block ab gives lane (j, g) the 4 consecutive
// antennas 16 ab + 4 g + r of RHS j, and the true-residual product
//   R[u][j] = sum_n H[u][n] x[n][j]
// reads them back as its B operand when the reduction index of chunk (ab,
// m) is ordered as antenna 16 ab + 4 kk + m for slot kk. Users are processed
// in VR-start order (perm), which keeps the nonzero tiles of the banded H
// and M few.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

struct MfmaLds {
    float2 *R;    // residual (greedy variants: the selection reads every row)
    float2 *PF;   // phi of the first step of an iteration (F rows, all rows, or one-hot)
    float2 *PV;   // phi of the aggregated V step; q at the confirm pass
    float2 *MP;   // one partial Gram product per part
    int *fpos;    // VALU half-step: sorted positions of the users of F
    float2 *MF;   // VALU half-step: the F columns of M, [row][f]
    float *nrm, *ninv, *pre, *red;   // ||a||^2 and 1 / ||a||^2 per sorted row
    int *posl;
    int *agoff, *gmoff;   // copies of the tile tables of this problem
    int *gmc;    // copy of the Gram chunk columns (at most nub * kpad / 4)
    int *gmnf;   // per row block: Gram chunks holding a user of F (a multiple of 4)
    int *rsel;   // per sorted row: 1 user of F, 2 user of V, 0 padding
    int *gidx;   // greedy: entry of the Gram chunk list of (row block, chunk), or -1: [nub][kpad / 4]
    int *selk;   // greedy: per column, the sorted position of the chosen row (-1: none)
    float2 *selg;   // greedy: per column, gamma of the chosen row
};

// Column state beyond the public flags: stopped on the maintained residual,
// waiting for the true residual to confirm.
constexpr int kPending = 8;
// Own entries per thread (EP) are at most this many: kpad <= kMaxEntries * 4 W.
constexpr int kMaxEntries = 4;

// Waves per 16-row block of the Gram product: the chunk groups of a block
// are split over nparts waves when there are more waves than blocks.
__host__ __device__ inline int gram_parts(int nub, int W)
{
    return nub <= W ? W / nub : 1;
}

__host__ __device__ inline size_t mfma_lds_layout(int kpad, int nab, int W, bool greedy, int nmf, char *base,
                                                  MfmaLds *L)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 15) & ~size_t(15);
        return base ? base + o : nullptr;
    };
    const size_t tile = (size_t)kpad * 16 * 8;
    char *R = take(greedy ? tile : 0);
    char *PF = take(greedy ? 0 : tile);   // the greedy step takes one Gram column, no operand
    char *PV = take(tile);
    char *MP = take(tile * gram_parts(kpad / 16, W));
    char *nrm = take((size_t)kpad * 4);
    char *ninv = take((size_t)kpad * 4);
    char *pre = take(greedy ? (size_t)W * kpad * 4 : 0);
    char *red = take((size_t)4 * W * 16 * 4);
    char *posl = take((size_t)kpad * 4);
    char *tabs = take((size_t)(nab + 1 + kpad / 16 + 1) * 4);
    char *gmc = take((size_t)(kpad / 16) * (kpad / 4 + 8) * 4);
    char *gmnf = take((size_t)(kpad / 16) * 4);
    char *rsel = take((size_t)kpad * 4);
    char *fpos = take(16 * 4);
    char *mf = take((size_t)kpad * nmf * 8);
    char *gidx = take(greedy ? (size_t)(kpad / 16) * (kpad / 4) * 4 : 0);
    char *selk = take(greedy ? 16 * 4 : 0);
    char *selg = take(greedy ? 16 * 8 : 0);
    // test the LDS base, not L: L points into a caller's register-resident
    // struct, and comparing its address would pin that struct to memory
    if (base) {
        int *tb = (int *)tabs;
        L->agoff = tb;
        L->gmoff = tb + nab + 1;
        L->gmc = (int *)gmc;
        L->gmnf = (int *)gmnf;
        L->R = (float2 *)R;
        L->PF = (float2 *)PF;
        L->PV = (float2 *)PV;
        L->MP = (float2 *)MP;
        L->nrm = (float *)nrm;
        L->ninv = (float *)ninv;
        L->pre = (float *)pre;
        L->red = (float *)red;
        L->posl = (int *)posl;
        L->rsel = (int *)rsel;
        L->fpos = (int *)fpos;
        L->MF = (float2 *)mf;
        L->gidx = (int *)gidx;
        L->selk = (int *)selk;
        L->selg = (float2 *)selg;
    }
    return off;
}

// Sums over the threads of each RHS column j = tid % 16; every thread gets
// its column's totals, added in a fixed order. One barrier: consecutive sums
// alternate between the two halves of the buffer (ColSums), so a sum never
// overwrites partials that a thread may still be reading from the previous
// one, and the sum before that was read before the previous barrier. Within
// a wave the four lanes of a column are added by col4_sum.
template <int W>
struct ColSums {
    float *red;   // 2 halves x 2 values x W waves x 16 columns
    int half;

    __device__ __forceinline__ float *next()
    {
        half ^= 1;
        return red + half * 2 * W * 16;
    }

    __device__ __forceinline__ float sum(float v)
    {
        const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
        float *b = next();
        v = col4_sum(v);
        if (lane < 16) b[w * 16 + lane] = v;
        __syncthreads();
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) s += b[i * 16 + (tid & 15)];
        return s;
    }

    __device__ __forceinline__ float2 sum2(float a, float c)
    {
        const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
        float *b = next();
        a = col4_sum(a);
        c = col4_sum(c);
        if (lane < 16) {
            b[w * 16 + lane] = a;
            b[(W + w) * 16 + lane] = c;
        }
        __syncthreads();
        float sa = 0.f, sc = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            sa += b[i * 16 + (tid & 15)];
            sc += b[(W + i) * 16 + (tid & 15)];
        }
        return float2{sa, sc};
    }
};

// Per-tile constants shared by the phases below (passed by value so that
// everything stays in registers after inlining).
using CDesc = const VRK_CONST VrkDesc;
template <typename T>
using gp = VRK_GLOBAL T *;

struct TileCtx {
    MfmaLds L;
    gp<const float2> S, HA, HG, GM;
    gp<float2> X;   // output rows of this tile's RHS (x = H^H q)
    gp<const int32_t> perm, ag_uc, gm_c;
    int64_t lds, ldx;
    int K, N, nub, kpad, nab, b0, nrhs, prob;
    float xi;
};

// H^H F on antenna block ab (F in LDS, [row][16]): chunks e of that block's
// list, four at a time so that their loads are in flight together.
__device__ __forceinline__ void agg_block(const TileCtx &c, int ab, const float2 *F, f4 &pr, f4 &pi)
{
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    C3 acc = c3_zero();
    const int e0 = c.L.agoff[ab], e1 = c.L.agoff[ab + 1];
    int e = e0;
#pragma unroll 1
    for (; e + 3 < e1; e += 4) {
        float2 h[4], f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            h[i] = c.HG[(int64_t)(e + i) * 64 + lane];
            f[i] = F[(4 * c.ag_uc[e + i] + g) * 16 + j];
        }
        // all four loads go out before the first wait (left alone, the
        // scheduler turns this into load, wait, MFMA per chunk)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) c3mfma(acc, h[i], f[i]);
    }
#pragma unroll 1
    for (; e < e1; ++e) c3mfma(acc, c.HG[(int64_t)e * 64 + lane], F[(4 * c.ag_uc[e] + g) * 16 + j]);
    c3_get(acc, pr, pi);
}

// x <- H^H q (every column) into the output rows: lane (j, g) of antenna
// block ab writes antennas 16 ab + 4 g .. + 3 of RHS b0 + j (two 16-byte
// stores when the row is 32-byte aligned).
template <int W>
__device__ __forceinline__ void form_x(const TileCtx &c)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int b = c.b0 + j;
    const gp<float2> row = c.X + (int64_t)(b < c.nrhs ? b : 0) * c.ldx;
#pragma unroll 1
    for (int ab = w; ab < c.nab; ab += W) {
        f4 qr, qi;
        agg_block(c, ab, c.L.PV, qr, qi);   // q, staged in PV
        const int n0 = 16 * ab + 4 * g;
        if (b < c.nrhs) {
            if (n0 + 3 < c.N && ((reinterpret_cast<uintptr_t>(row + n0) & 31) == 0)) {
                *(gp<float4>)(row + n0) = float4{qr[0], qi[0], qr[1], qi[1]};
                *(gp<float4>)(row + n0 + 2) = float4{qr[2], qi[2], qr[3], qi[3]};
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (n0 + r < c.N) row[n0 + r] = float2{qr[r], qi[r]};
            }
        }
    }
}

// Gram work of a wave: with nub <= W, wave w < nparts * nub takes chunk
// groups [g0, g1) of row block mb = w % nub as part w / nub; with more blocks
// than waves it takes the whole blocks w, w + W, ... The first GR chunks of
// its first block sit in registers for an iteration phase (tiles and their
// chunk columns), loaded by gram_load.
template <int GR>
struct GramRegs {
    float2 m[GR > 0 ? GR : 1];
    int uc[GR > 0 ? GR : 1];
    int mb, part, g0, g1;
};

template <int W, int GR>
__device__ __forceinline__ void gram_load(const TileCtx &c, GramRegs<GR> &gr)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int np = gram_parts(c.nub, W);
    gr.mb = -1;
    gr.part = 0;
    gr.g0 = gr.g1 = 0;
    if (c.nub <= W) {
        if (w < np * c.nub) {
            gr.mb = w % c.nub;
            gr.part = w / c.nub;
            const int ng = (c.L.gmoff[gr.mb + 1] - c.L.gmoff[gr.mb]) / 4;
            gr.g0 = gr.part * ng / np;
            gr.g1 = (gr.part + 1) * ng / np;
        }
    } else if (w < c.nub) {
        gr.mb = w;
        gr.g1 = (c.L.gmoff[w + 1] - c.L.gmoff[w]) / 4;
    }
    const int e0 = gr.mb >= 0 ? c.L.gmoff[gr.mb] + 4 * gr.g0 : 0;
    const int n = 4 * (gr.g1 - gr.g0);
#pragma unroll
    for (int q = 0; q < GR; ++q) {
        gr.m[q] = float2{0.f, 0.f};
        gr.uc[q] = 0;
        if (q < n) {
            gr.m[q] = c.GM[(int64_t)(e0 + q) * 64 + lane];
            gr.uc[q] = __builtin_amdgcn_readfirstlane(c.L.gmc[e0 + q]);
        }
    }
}

// Four chunks e .. e + 3 of a row block from memory: loads first, then MFMAs.
__device__ __forceinline__ void gram_group(const TileCtx &c, const float2 *F, int e, C3 &acc)
{
    const int lane = threadIdx.x & 63;
    float2 m[4], f[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        m[i] = c.GM[(int64_t)(e + i) * 64 + lane];
        f[i] = F[c.L.gmc[e + i] * 64 + lane];   // row 4 uc + g, column j
    }
    __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
    for (int i = 0; i < 4; ++i) c3mfma(acc, m[i], f[i]);
}

// Partial Gram products of the wave's work: the MFMA result (rows
// 16 mb + 4 g + r, column j) of its chunks of M F goes to the part's slice
// MP[part] of LDS. Parts are summed by the element-wise pass after a barrier.
// With fonly, only the groups covering the chunks that hold users of F
// (listed first) are taken: F is zero on every other row. Returns the
// lane's share of F^H (M F) for its column (0 unless with_den), so the
// column sum of the returns over the workgroup is phi^H M phi.
template <int W, int GR>
__device__ __forceinline__ float gram_part(const TileCtx &c, const float2 *F, const GramRegs<GR> &gr, bool fonly,
                                           bool with_den)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    float den = 0.f;
    auto block = [&](int mb, int g0, int g1, bool regs) {
        if (fonly) g1 = min(g1, (c.L.gmnf[mb] + 3) / 4);
        C3 acc = c3_zero();
        const int e0 = c.L.gmoff[mb];
        int gg = g0;
        if (regs) {
#pragma unroll
            for (int q4 = 0; q4 < GR / 4; ++q4)
                if (g0 + q4 < g1) {
                    float2 f[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) f[i] = F[gr.uc[4 * q4 + i] * 64 + lane];
#pragma unroll
                    for (int i = 0; i < 4; ++i) c3mfma(acc, gr.m[4 * q4 + i], f[i]);
                }
            gg = g0 + GR / 4;
        }
#pragma unroll 1
        for (; gg < g1; ++gg) gram_group(c, F, e0 + 4 * gg, acc);
        f4 mr, mi;
        c3_get(acc, mr, mi);
        float2 *out = c.L.MP + (size_t)(regs ? gr.part : 0) * c.kpad * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * mb + 4 * g + r;
            out[row * 16 + j] = float2{mr[r], mi[r]};
            if (with_den) {
                const float2 f = F[row * 16 + j];
                den += f.x * mr[r] + f.y * mi[r];
            }
        }
    };
    if (c.nub <= W) {
        if (gr.mb >= 0) block(gr.mb, gr.g0, gr.g1, true);
    } else {
#pragma unroll 1
        for (int mb = w; mb < c.nub; mb += W)
            block(mb, 0, (c.L.gmoff[mb + 1] - c.L.gmoff[mb]) / 4, mb == w);
    }
    return den;
}

// Right-hand side of the adjoint solve, b = H g, for this tile's RHS:
// partial products like the Gram parts (wave w takes row block w % nub and
// part w / nub of its antenna-block range, or whole blocks w, w + W, ...),
// H from the residual tiles (16 users x antennas 16 ab + 4 kk + m at lane
// i + 16 kk), g from the rows of GX as the B operand (4 consecutive
// antennas per lane), results to MP[part]. A barrier must precede reading MP.
template <int W>
__device__ __forceinline__ void hg_part(const TileCtx &c, CDesc &d)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int b = c.b0 + j;
    const gp<const float2> grow = gmem(static_cast<const float2 *>(d.GX)) + (int64_t)(b < c.nrhs ? b : 0) * d.ldgx;
    auto block = [&](int mb, int part, int np) {
        const int lo = gmem(d.rab_lo)[mb], hi = gmem(d.rab_hi)[mb];
        const int64_t hb = gmem(d.ha_off)[mb];
        const int a0 = lo + part * (hi - lo) / np, a1 = lo + (part + 1) * (hi - lo) / np;
        C3 acc = c3_zero();
        // four antenna blocks per step: their loads are in flight together
#pragma unroll 1
        for (int ab0 = a0; ab0 < a1; ab0 += 4) {
            float2 h[4][4], x[4][4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int ab = ab0 + t;
                const gp<const float2> hp = c.HA + (hb + 4 * (int64_t)(ab - lo)) * 64 + lane;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int n = 16 * ab + 4 * g + m;
                    h[t][m] = x[t][m] = float2{0.f, 0.f};
                    if (ab < a1) {
                        h[t][m] = hp[64 * m];
                        if (b < c.nrhs && n < c.N) x[t][m] = grow[n];
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);   // all loads in flight before the first wait
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int m = 0; m < 4; ++m) c3mfma(acc, h[t][m], x[t][m]);
        }
        f4 mr, mi;
        c3_get(acc, mr, mi);
        float2 *out = c.L.MP + (size_t)part * c.kpad * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(16 * mb + 4 * g + r) * 16 + j] = float2{mr[r], mi[r]};
    };
    if (c.nub <= W) {
        const int np = gram_parts(c.nub, W);
        if (w < np * c.nub) block(w % c.nub, w / c.nub, np);
    } else {
#pragma unroll 1
        for (int mb = w; mb < c.nub; mb += W) block(mb, 0, 1);
    }
}

// Sum of the partial Gram products at entry (ku, j).
__device__ __forceinline__ float2 gram_sum(const TileCtx &c, int np, int ku, int j)
{
    float2 s = {0.f, 0.f};
#pragma unroll 4
    for (int p = 0; p < np; ++p) {
        const float2 v = c.L.MP[((size_t)p * c.kpad + ku) * 16 + j];
        s.x += v.x;
        s.y += v.y;
    }
    return s;
}

template <int W, int EP, int VARIANT>
__device__ __forceinline__ void solve_item(const VrkSolveArgs &a, const int prob, const int tile, char *smem)
{
    // prob and tile are wave-uniform, so the descriptor is read with scalar loads
    CDesc &d = ((CDesc *)a.desc)[prob];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, j = lane & 15;
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
    constexpr int variant = VARIANT;
    constexpr bool greedy = variant == 0 || variant == 2;
    mfma_lds_layout(c.kpad, c.nab, W, greedy, d.nmf, smem, &c.L);
    const MfmaLds &L = c.L;
    gp<float2> X, V;
    int64_t ldx_, ldv_;
    if (a.adjoint) {
        c.S = nullptr; c.lds = 0;   // b = H g is formed by the tile itself
        X = nullptr; ldx_ = 0;      // H^H mu is not formed
        V = gmem(static_cast<float2 *>(d.GS)); ldv_ = d.ldgs;
    } else {
        c.S = gmem(static_cast<const float2 *>(d.S)); c.lds = d.lds;
        X = gmem(static_cast<float2 *>(d.X)); ldx_ = d.ldx;
        V = gmem(static_cast<float2 *>(d.V)); ldv_ = d.ldv;
    }
    c.HA = gmem(static_cast<const float2 *>(d.HA));
    c.HG = gmem(static_cast<const float2 *>(d.HG));
    c.GM = gmem(static_cast<const float2 *>(d.GM));
    c.X = X;
    c.ldx = ldx_;
    c.perm = gmem(d.perm);
    c.ag_uc = gmem(d.ag_uc);
    c.gm_c = gmem(d.gm_c);
    const gp<const float> nrm_g = gmem(static_cast<const float *>(d.nrm));
    const int K = c.K, kpad = c.kpad, b0 = c.b0;
    const int rows_per_pass = W * 4;   // (row, column) entries: tid -> (tid / 16, tid % 16)
    const int er = tid >> 4;

    // ---- init: tables in LDS, then q = 0, r = s (z0 = 0), norms in VR-start order
    for (int ku = tid; ku < kpad; ku += W * 64) {
        L.nrm[ku] = ku < K ? nrm_g[c.perm[ku]] : 1.f;
        L.ninv[ku] = 1.f / L.nrm[ku];
        L.rsel[ku] = ku < K ? (gmem(d.inf)[c.perm[ku]] ? 1 : 2) : 0;
        if (ku < K) L.posl[c.perm[ku]] = ku;
    }
    for (int i = tid; i <= c.nab; i += W * 64) L.agoff[i] = gmem(d.ag_off)[i];
    for (int i = tid; i <= c.nub; i += W * 64) L.gmoff[i] = gmem(d.gm_off)[i];
    for (int i = tid; i < gmem(d.gm_off)[c.nub]; i += W * 64) L.gmc[i] = max(c.gm_c[i], 0);   // padding: zero tile
    for (int i = tid; i < c.nub; i += W * 64) L.gmnf[i] = gmem(d.gm_nf)[i];
    if (greedy) {
        // (row block, chunk) -> entry of the block's Gram chunk list
        for (int i = tid; i < c.nub * (kpad / 4); i += W * 64) L.gidx[i] = -1;
        __syncthreads();
        for (int mb = 0; mb < c.nub; ++mb) {
            const int e0 = gmem(d.gm_off)[mb], e1 = gmem(d.gm_off)[mb + 1];
            for (int e = e0 + tid; e < e1; e += W * 64) {
                const int uc = c.gm_c[e];
                if (uc >= 0) L.gidx[mb * (kpad / 4) + uc] = e;
            }
        }
    }
    // > 0: VALU orthogonal half-step from MF (never with four entries per
    // thread: its registers are needed elsewhere)
    const int nmf = EP >= 4 ? 0 : d.nmf;
    if (tid < nmf) L.fpos[tid] = gmem(d.fpos)[tid];
    for (int i = tid; i < kpad * nmf; i += W * 64) L.MF[i] = gmem(static_cast<const float2 *>(d.MF))[i];
    __syncthreads();
    // adjoint: b = H g for this tile's columns
    const int np = c.nub <= W ? gram_parts(c.nub, W) : 1;
    if (a.adjoint) {
        hg_part<W>(c, d);
        __syncthreads();
    }
    // this thread's entries (ku, j), ku = er + rows_per_pass k: residual,
    // dual iterate, phi; with up to two entries per thread also the
    // right-hand side, 1 / ||a_ku||^2 and the F/V selector (with four, those
    // are read again when needed: the right-hand side from S, or, in the
    // adjoint solve, from the VR-start-order output rows that hold b until
    // mu goes there)
    constexpr bool lean = EP >= 4;
    float2 rr[EP], qq[EP], pp[EP];
    float2 sb[lean ? 1 : EP];
    float ninv[lean ? 1 : EP];
    int rs[lean ? 1 : EP];
    auto own = [&](int k) { return er + rows_per_pass * k; };
    auto sel = [&](int k) { return lean ? (own(k) < kpad ? L.rsel[own(k)] : 0) : rs[k]; };
    auto inv_norm = [&](int k) { return lean ? L.ninv[own(k)] : ninv[k]; };
    const gp<float2> bkeep = gmem(static_cast<float2 *>(d.Msrt));
    auto rhs = [&](int k) -> float2 {
        if (!lean) return sb[k];
        const int ku = own(k), b = b0 + j;
        if (b >= c.nrhs) return float2{0.f, 0.f};
        if (a.adjoint) return bkeep[(int64_t)b * kpad + ku];
        float2 v = {0.f, 0.f};
        if (ku < K) v = c.S[(int64_t)b * c.lds + c.perm[ku]];
        return v;
    };
    // phi for the first step of an iteration: rows of F (VR-OAHK), every
    // row (AHK), none (greedy variants: one-hot, written by the selection)
    auto phi_first = [&](int k) -> float2 {
        const int rsk = sel(k);
        const bool in = variant == 1 ? rsk != 0 : (variant == 3 ? rsk == 1 : false);
        const float f = in ? inv_norm(k) : 0.f;
        return float2{rr[k].x * f, rr[k].y * f};
    };
    ColSums<W> cs{L.red, 0};
    float r2 = 0.f, num = 0.f;
#pragma unroll
    for (int k = 0; k < EP; ++k) {
        const int ku = own(k);
        rr[k] = qq[k] = pp[k] = float2{0.f, 0.f};
        if (!lean) {
            sb[k] = float2{0.f, 0.f};
            ninv[k] = 0.f;
            rs[k] = 0;
        }
        if (ku < kpad) {
            const int b = b0 + j;
            float2 s0 = {0.f, 0.f};
            if (a.adjoint) {
                s0 = gram_sum(c, np, ku, j);
                if (lean && b < c.nrhs) bkeep[(int64_t)b * kpad + ku] = s0;
            } else if (ku < K && b < c.nrhs) {
                s0 = c.S[(int64_t)b * c.lds + c.perm[ku]];
            }
            rr[k] = s0;
            if (!lean) {
                sb[k] = s0;
                rs[k] = L.rsel[ku];
                ninv[k] = L.ninv[ku];
            }
            pp[k] = phi_first(k);
            if (!greedy) L.PF[ku * 16 + j] = pp[k];
            if (greedy) L.R[ku * 16 + j] = rr[k];
            r2 += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
            num += pp[k].x * rr[k].x + pp[k].y * rr[k].y;
        }
    }
    {
        const float2 t = cs.sum2(r2, num);
        r2 = t.x;
        num = t.y;
    }
    const float fro2 = *gmem(static_cast<const float *>(d.fro2));
    // state of this thread's column j, identical in every thread of the column
    const float sn = sqrtf(r2);
    bool act = false;
    int fl = 0, its = 0;
    float rel = 0.f;
    if (b0 + j < c.nrhs) {
        if (!isfinite(sn) || !isfinite(fro2)) fl = VRK_FLAG_NONFINITE;
        else if (r2 == 0.f) fl = VRK_FLAG_CONVERGED;
        else act = true;
    }

    // Gram tiles kept in registers per wave (two VGPRs and a chunk column each)
    constexpr int GR = W == 8 ? 16 : (EP >= 2 ? 0 : 4);
    int64_t t_it = 0;
    for (;;) {
        // iteration phase: runs until every column has stopped
        GramRegs<GR> gr;
        gram_load<W, GR>(c, gr);
        for (;;) {
            // stop rule on the maintained residual, every check_every
            // iterations and at the cap
            if (act && (a.check_every == 1 || t_it % a.check_every == 0 || t_it >= a.max_iters)) {
                rel = sqrtf(r2) / sn;
                its = (int)t_it;
                if (!isfinite(rel)) { fl = VRK_FLAG_NONFINITE; act = false; }
                else if (rel <= (float)a.tol) { fl = kPending; act = false; }
                else if (t_it >= a.max_iters) { fl = VRK_FLAG_MAXITER; act = false; }
            }
            if (__ballot(act) == 0) break;   // lanes 0..15 of a wave hold all 16 columns

            if constexpr (greedy) {
                // greedy selection, one wave per column, from the residuals in
                // LDS: column cc projects onto row i with gamma = r_i / ||a_i||^2.
                // In the dual that step is q_i += gamma, r -= gamma M[:, i]: only
                // the rows of X_i change (Theorem 2: M[:, i] is zero elsewhere),
                // taken from the one Gram tile column holding i per row block.
                for (int cc = w; cc < 16; cc += W) {
                    if (!__shfl(act, cc, 64)) {
                        if (lane == 0) L.selk[cc] = -1;
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
                        const float2 r = L.R[ku * 16 + cc];
                        L.selk[cc] = ku;
                        L.selg[cc] = float2{r.x * inv, r.y * inv};
                    }
                }
                __syncthreads();
                const int kp = L.selk[j];
                const float2 gmv = L.selg[j];
                r2 = 0.f;
#pragma unroll
                for (int k = 0; k < EP; ++k) {
                    const int ku = own(k);
                    if (ku < kpad) {
                        if (kp >= 0) {
                            const int e = L.gidx[(ku >> 4) * (kpad / 4) + (kp >> 2)];
                            if (e >= 0) {
                                const float2 m = c.GM[(int64_t)e * 64 + (ku & 15) + 16 * (kp & 3)];
                                rr[k] = float2{rr[k].x - (m.x * gmv.x - m.y * gmv.y),
                                               rr[k].y - (m.x * gmv.y + m.y * gmv.x)};
                            }
                            if (ku == kp) qq[k] = float2{qq[k].x + gmv.x, qq[k].y + gmv.y};
                            L.R[ku * 16 + j] = rr[k];
                        }
                        r2 += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
                    }
                }
                r2 = cs.sum(r2);
            } else if constexpr (variant == 1) {
                // aggregated step over all rows: phi = PF, num known; the
                // Gram waves add phi^H M phi as they go
                const float den = cs.sum(gram_part<W, GR>(c, L.PF, gr, false, true));
                const float gm = (act && num > 0.f && den > 0.f) ? num / den : 0.f;
                r2 = 0.f;
                float nn = 0.f;
#pragma unroll
                for (int k = 0; k < EP; ++k) {
                    const int ku = own(k);
                    if (ku < kpad) {
                        const float2 m = gram_sum(c, np, ku, j);
                        qq[k] = float2{qq[k].x + gm * pp[k].x, qq[k].y + gm * pp[k].y};
                        rr[k] = float2{rr[k].x - gm * m.x, rr[k].y - gm * m.y};
                        pp[k] = phi_first(k);
                        L.PF[ku * 16 + j] = pp[k];
                        r2 += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
                        nn += pp[k].x * rr[k].x + pp[k].y * rr[k].y;
                    }
                }
                const float2 t = cs.sum2(r2, nn);
                r2 = t.x;
                num = t.y;
            } else {
                // orthogonal half-step on F with gamma = 1 (Prop. 1): q_F += phi_F,
                // r -= M phi_F (the F columns of M); then phi_V of the new residual
                const bool hasv = d.nv > 0;
                if (nmf == 0) {
                    gram_part<W, GR>(c, L.PF, gr, true, false);
                    __syncthreads();
                }
                float nv_num = 0.f;
                r2 = 0.f;
#pragma unroll
                for (int k = 0; k < EP; ++k) {
                    const int ku = own(k);
                    if (ku < kpad) {
                        float2 m = {0.f, 0.f};
                        if (nmf == 0) {
                            m = gram_sum(c, np, ku, j);
                        } else {
                            // VALU: sum over the users of F of M[ku][f] phi_F[f]
                            const float2 *mrow = L.MF + ku * nmf;
#pragma unroll 4
                            for (int t = 0; t < nmf; ++t) {
                                const float2 mv = mrow[t], f = L.PF[L.fpos[t] * 16 + j];
                                m.x += mv.x * f.x - mv.y * f.y;
                                m.y += mv.x * f.y + mv.y * f.x;
                            }
                        }
                        if (act) {
                            qq[k] = float2{qq[k].x + pp[k].x, qq[k].y + pp[k].y};
                            rr[k] = float2{rr[k].x - m.x, rr[k].y - m.y};
                        }
                        // phi of the next step: rows of V for the aggregated
                        // step, or, without V, rows of F for the next iteration
                        const float f = sel(k) == (hasv ? 2 : 1) ? inv_norm(k) : 0.f;
                        pp[k] = float2{rr[k].x * f, rr[k].y * f};
                        (hasv ? L.PV : L.PF)[ku * 16 + j] = pp[k];
                        nv_num += pp[k].x * rr[k].x + pp[k].y * rr[k].y;
                        r2 += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
                    }
                }
                if (!hasv) {
                    r2 = cs.sum(r2);
                } else {
                    // aggregated step on V: gamma = phi^H r / phi^H M phi
                    __syncthreads();
                    const float den = gram_part<W, GR>(c, L.PV, gr, false, true);
                    const float2 nd = cs.sum2(nv_num, den);
                    const float gm = (act && nd.x > 0.f && nd.y > 0.f) ? nd.x / nd.y : 0.f;
                    r2 = 0.f;
#pragma unroll
                    for (int k = 0; k < EP; ++k) {
                        const int ku = own(k);
                        if (ku < kpad) {
                            const float2 m = gram_sum(c, np, ku, j);
                            qq[k] = float2{qq[k].x + gm * pp[k].x, qq[k].y + gm * pp[k].y};
                            rr[k] = float2{rr[k].x - gm * m.x, rr[k].y - gm * m.y};
                            pp[k] = phi_first(k);
                            L.PF[ku * 16 + j] = pp[k];
                            r2 += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
                        }
                    }
                    r2 = cs.sum(r2);
                }
            }
            ++t_it;
        }
        // every column stopped: x = H^H q goes out, and the residual
        // s - A A^H q = s - M q, evaluated afresh from q (free of the drift
        // of the maintained residual), decides
#pragma unroll
        for (int k = 0; k < EP; ++k)
            if (own(k) < kpad) L.PV[own(k) * 16 + j] = qq[k];
        __syncthreads();
        if (!a.adjoint) form_x<W>(c);   // the gradient products need no H^H mu
        gram_part<W, GR>(c, L.PV, gr, false, false);
        __syncthreads();
        float t2 = 0.f, tn = 0.f;
#pragma unroll
        for (int k = 0; k < EP; ++k) {
            const int ku = own(k);
            if (ku < kpad) {
                const float2 mq = gram_sum(c, np, ku, j);
                const float2 s0 = rhs(k);
                rr[k] = float2{s0.x - mq.x, s0.y - mq.y};
                if (greedy) L.R[ku * 16 + j] = rr[k];
                pp[k] = phi_first(k);
                if (!greedy) L.PF[ku * 16 + j] = pp[k];
                t2 += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
                tn += pp[k].x * rr[k].x + pp[k].y * rr[k].y;
            }
        }
        {
            const float2 t = cs.sum2(t2, tn);
            t2 = t.x;
            tn = t.y;
        }
        // columns stopped by the rule or the iteration cap take the true
        // residual's verdict; a column it rejects resumes while the cap allows
        if (fl == kPending || fl == VRK_FLAG_MAXITER) {
            rel = sqrtf(t2) / sn;
            if (!isfinite(rel)) fl = VRK_FLAG_NONFINITE;
            else if (rel <= (float)a.tol) fl = VRK_FLAG_CONVERGED;
            else if (t_it < a.max_iters) { fl = 0; act = true; }
            else fl = VRK_FLAG_MAXITER;
        }
        if (__ballot(act) == 0) break;
        r2 = t2;   // the resumed columns go on from the true residual
        num = tn;
    }

    // ---- outputs: x is in place (form_x, forward only); v (or mu) in caller order and in
    // VR-start order for the gradient products
    {
        // the column and the first row made opaque here, so that the output
        // addresses are formed now rather than kept live (spilled) from init
        int jq = j, eq = er;
        asm volatile("" : "+v"(jq), "+v"(eq));
        const int b = b0 + jq;
        if (b < c.nrhs) {
            const gp<float2> VS = gmem(static_cast<float2 *>(a.adjoint ? d.Msrt : d.Vsrt));
#pragma unroll
            for (int k = 0; k < EP; ++k) {
                const int ku = eq + rows_per_pass * k;
                if (V && ku < K) V[(int64_t)b * ldv_ + c.perm[ku]] = qq[k];
                if (VS && ku < kpad) VS[(int64_t)b * kpad + ku] = qq[k];
            }
        }
    }
    if (tid < 16) {
        const int b = b0 + tid;
        if (b < c.nrhs) {
            const int64_t gidx = d.rhs_base + b;
            if (a.iters) gmem(a.iters)[gidx] = its;
            if (a.relres) gmem(a.relres)[gidx] = rel;
            if (a.flags) gmem(a.flags)[gidx] = fl;
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

template <int W, int EP, int VARIANT, bool PERSIST>
__global__ void __launch_bounds__(W * 64) k_mfma_solve(VrkSolveArgs a, const VrkWork *work, VrkQueue q)
{
    extern __shared__ __align__(16) char smem[];
    if constexpr (!PERSIST) {
        const VrkWork wk = gmem(work)[blockIdx.x];   // one workgroup per work item
        solve_item<W, EP, VARIANT>(a, __builtin_amdgcn_readfirstlane(wk.prob),
                                   __builtin_amdgcn_readfirstlane(wk.tile), smem);
    } else {
        __shared__ int sh_item;
        for (int item = next_item(q, &sh_item); item >= 0; item = next_item(q, &sh_item)) {
            const VrkWork wk = gmem(work)[item];
            solve_item<W, EP, VARIANT>(a, __builtin_amdgcn_readfirstlane(wk.prob),
                                       __builtin_amdgcn_readfirstlane(wk.tile), smem);
        }
    }
}

__global__ void k_queue_reset(int *count)
{
    if (threadIdx.x < VRK_NQUEUE) count[threadIdx.x] = 0;
}

// Launch (mode 0), set the LDS attribute and report occupancy (mode 1).
template <int W, int EP, int VARIANT, bool PERSIST>
hipError_t launch_kernel(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid,
                         size_t lds, hipStream_t s, int mode, int *blocks_per_cu)
{
    auto kern = k_mfma_solve<W, EP, VARIANT, PERSIST>;
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

template <int W, int EP, int VARIANT>
hipError_t launch_one(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid, size_t lds,
                      hipStream_t s, int mode, int *blocks_per_cu)
{
    if (q.count) return launch_kernel<W, EP, VARIANT, true>(a, work, q, grid, lds, s, mode, blocks_per_cu);
    return launch_kernel<W, EP, VARIANT, false>(a, work, q, grid, lds, s, mode, blocks_per_cu);
}

// GRK and VR-OGRK share one kernel: in the dual space the Gram column's
// sparsity already confines each update to X_pick.
template <int W, int EP>
hipError_t launch_variant(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid, size_t lds,
                          hipStream_t s, int mode, int *bpc)
{
    switch (a.variant) {
    case 0:
    case 2: return launch_one<W, EP, 0>(a, work, q, grid, lds, s, mode, bpc);
    case 1: return launch_one<W, EP, 1>(a, work, q, grid, lds, s, mode, bpc);
    case 3: return launch_one<W, EP, 3>(a, work, q, grid, lds, s, mode, bpc);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int vrk_mfma_entries(int32_t kpad, int32_t waves)
{
    if (waves != 8 && waves != 16) return 0;
    const int need = (kpad + 4 * waves - 1) / (4 * waves);
    int ep = 1;
    while (ep < need) ep *= 2;
    return ep <= kMaxEntries ? ep : 0;
}

int vrk_mfma_supported(int32_t kpad, int32_t waves)
{
    return vrk_mfma_entries(kpad, waves) > 0;
}

size_t vrk_mfma_lds_bytes(int32_t kpad, int32_t nab, int32_t waves, int32_t greedy, int32_t nmf)
{
    return mfma_lds_layout(kpad, nab, waves, greedy != 0, nmf, nullptr, nullptr);
}

hipError_t vrk_launch_mfma_solve(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid,
                                 int32_t waves, int32_t ep, size_t lds, hipStream_t s, int mode, int *bpc)
{
    if (grid <= 0) return hipSuccess;
#define VRK_EP_CASES(W)                                                          \
    switch (ep) {                                                                \
    case 1: return launch_variant<W, 1>(a, work, q, grid, lds, s, mode, bpc);    \
    case 2: return launch_variant<W, 2>(a, work, q, grid, lds, s, mode, bpc);    \
    case 4: return launch_variant<W, 4>(a, work, q, grid, lds, s, mode, bpc);    \
    }
    if (waves == 8) {
        VRK_EP_CASES(8)
    } else if (waves == 16) {
        VRK_EP_CASES(16)
    }
#undef VRK_EP_CASES
    return hipErrorInvalidValue;
}
