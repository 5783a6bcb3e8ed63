// Wave-owned MFMA engine for the aggregated sweeps (AHK, VR-OAHK): one
// workgroup of T waves per tile of 16 right-hand sides sharing a channel,
// several tiles per compute unit.
//
// Same dual-space iteration as the block engine (mfma_engine.hip): from
// z = 0 every step keeps x = H^H q, so the residual is r = s - M q with
// M = H H^H + xi I, and an aggregated step r -= gamma M phi, q += gamma phi
// (eq. update4 with the coefficient of eq. coefficient, phi_i = r_i /
// ||a_i||^2 on the step's rows; Prop. 1's orthogonal half-step on F has
// gamma = 1 and only the F columns of M). The layout differs: the 16-user
// row blocks of the tile are owned by the waves (wave w owns blocks w,
// w + T, ...), and each wave keeps r, q and its products in registers in the
// matrix cores' own output layout: lane (j, g) = (lane % 16, lane / 16) holds
// users 16 mb + 4 g + 0..3 of RHS column j (users in VR-start order). A Gram
// product over the block's chunk list (tiles of M, 16 users x 4 users) lands
// directly in the owner's registers; only phi travels through LDS, as the B
// operand of every wave's products. Per iteration the waves of a tile meet at
// three barriers (two for AHK) for the column sums ||r||^2, phi^H r and
// phi^H M phi; a tile has few waves, so other tiles on the same compute unit
// keep the matrix cores busy while one waits. q (touched once per step) and
// the row scales 1 / ||a_i||^2 live in LDS, which keeps the registers to r
// and one product per owned row.
//
// When every column has met the stop rule, x = H^H q goes to the output rows
// and the residual s - M q is evaluated afresh from q (free of the
// maintained residual's drift); a column it rejects resumes from it.
//
// The adjoint solve forms its right-hand side b = H g per owned block from
// the residual tiles (the product's output layout is the state layout), and
// keeps it in the VR-start-order rows of Msrt until mu replaces it.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

using CDesc = const VRK_CONST VrkDesc;
template <typename T>
using gp = VRK_GLOBAL T *;
template <typename T>
using cp = const VRK_CONST T *;

// Column state beyond the public flags: stopped on the maintained residual,
// waiting for the fresh residual to confirm.
constexpr int kPending = 8;

struct WLds {
    float2 *PV;   // phi of the aggregated step (all rows): [row][16]
    float2 *Q;    // the dual iterate q: [row][16]; each entry is touched by its owner lane
                  // only, except as the operand of x = H^H q and M q at the confirm pass
    float2 *PF;   // VR-OAHK: phi of the orthogonal half-step, the chunks holding users of F:
                  // [slot][64]; slot VRK_WAVE_FCHUNKS stays zero (the operand of other chunks)
    int *fslot;   // VR-OAHK: chunk -> slot in PF, or VRK_WAVE_FCHUNKS
    float *fv;    // per row: 1 / ||a||^2 on the rows of the aggregated step, else 0
    float *ff;    // per row (VR-OAHK): 1 / ||a||^2 on the rows of F, else 0
    float *red;   // column-sum partials: [3 sums][2 values][T waves][16 columns]
};

__host__ __device__ inline size_t wave_lds_layout(int kpad, int T, bool oahk, char *base, WLds *L)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 15) & ~size_t(15);
        return base ? base + o : nullptr;
    };
    char *pv = take((size_t)kpad * 16 * 8);
    char *q = take((size_t)kpad * 16 * 8);
    char *pf = take(oahk ? (size_t)(VRK_WAVE_FCHUNKS + 1) * 64 * 8 : 0);
    char *fs = take(oahk ? (size_t)(kpad / 4) * 4 : 0);
    char *fv = take((size_t)kpad * 4);
    char *ff = take(oahk ? (size_t)kpad * 4 : 0);
    char *red = take((size_t)3 * 2 * T * 16 * 4);
    if (base) {
        L->PV = (float2 *)pv;
        L->Q = (float2 *)q;
        L->PF = (float2 *)pf;
        L->fslot = (int *)fs;
        L->fv = (float *)fv;
        L->ff = (float *)ff;
        L->red = (float *)red;
    }
    return off;
}

// Sums over the 16 RHS columns of the tile: the four lanes of a column in
// each wave by row-swap moves, then the T waves' partials through LDS slot
// `slot` (one barrier), added in wave order; every lane gets its column's
// totals. Slots are distinct per call site in an iteration, so a slot is
// written again only after two more barriers.
template <int T, int NV>
__device__ __forceinline__ void colsum(float (&v)[NV], float *red, int slot)
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, j = lane & 15;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = col4_sum(v[i]);
    if constexpr (T == 1) {
        __syncthreads();   // also publishes this wave's LDS writes to its other lanes
    } else {
        float *b = red + slot * 2 * T * 16;
        if (lane < 16)
#pragma unroll
            for (int i = 0; i < NV; ++i) b[(i * T + w) * 16 + j] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < T; ++t) s += b[(i * T + t) * 16 + j];
            v[i] = s;
        }
    }
}

// Product of one owned row block with the B operand in LDS: the block's
// chunk entries [e0, e1) (a multiple of four; padding entries hold zero
// tiles), tile e of M at GM[64 e + lane] times chunk idx[e] of the operand
// (the entry's chunk, gm_c; or for the compact PF buffer of F chunks its
// slot there, gm_fs, whose spare slot is zero for other chunks). Only the
// entries before e_real contribute (the others are padding, at the end of
// the list): whole groups of four run without branches, software-pipelined
// (the tiles of the next group in flight while the current one is
// multiplied); the last group, when e_real cuts it, skips the products of
// its padding entries.
__device__ __forceinline__ void block_product(gp<const float2> GM, cp<int32_t> idx, int e0, int e_real,
                                              const float2 *B, f4 &pr, f4 &pi)
{
    const int lane = threadIdx.x & 63;
    C3 acc = c3_zero();
    auto operand = [&](int e) -> float2 {
        const int c = __builtin_amdgcn_readfirstlane(idx[e]);
        return B[(c > 0 ? c : 0) * 64 + lane];
    };
    const int ef = e0 + ((e_real - e0) & ~3);   // end of the whole groups
    const int eg = ef < e_real ? ef + 4 : ef;   // end of the groups loaded
    float2 m[4], mn[4];
    if (e0 < eg) {
#pragma unroll
        for (int i = 0; i < 4; ++i) m[i] = GM[(int64_t)(e0 + i) * 64 + lane];
    }
#pragma unroll 1
    for (int e = e0; e < ef; e += 4) {
        const bool more = e + 4 < eg;
        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i) mn[i] = GM[(int64_t)(e + 4 + i) * 64 + lane];
        }
        float2 f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = operand(e + i);
#pragma unroll
        for (int i = 0; i < 4; ++i) c3mfma(acc, m[i], f[i]);
        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i) m[i] = mn[i];
        }
    }
    if (ef < e_real) {
        float2 f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = operand(ef + i);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (ef + i < e_real) c3mfma(acc, m[i], f[i]);
    }
    c3_get(acc, pr, pi);
}

// End of the real entries of a chunk list [e0, e1): the padding (-1) entries
// close it, at most three (the lists are padded to a multiple of four).
__device__ __forceinline__ int list_real_end(cp<int32_t> idx, int e0, int e1)
{
    int e = e1;
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (e > e0 && __builtin_amdgcn_readfirstlane(idx[e - 1]) < 0) --e;
    return e;
}

template <int T, int BPW, int VARIANT>
__device__ __forceinline__ void wave_item(const VrkSolveArgs &a, const int prob, const int tile, char *smem)
{
    CDesc &d = ((CDesc *)a.desc)[prob];
    constexpr bool oahk = VARIANT == 3;
    // the wave index is uniform: in a scalar register, so the branches on
    // owned blocks are scalar
    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, j = lane & 15,
              g = lane >> 4;
    const int K = d.k, nub = d.nub, kpad = nub * VRK_UB, nab = d.nab, N = d.nt;
    const int b0 = tile * VRK_TILE_RHS, nrhs = d.nrhs, b = b0 + j;
    const bool colok = b < nrhs;
    WLds L;
    wave_lds_layout(kpad, T, oahk, smem, &L);
    const gp<const float2> GM = gmem(static_cast<const float2 *>(d.GM));
    const gp<const int32_t> perm = gmem(d.perm);
    const cp<int32_t> gmoff = (cp<int32_t>)d.gm_off, gmc = (cp<int32_t>)d.gm_c, gmnf = (cp<int32_t>)d.gm_nf,
                      gmfs = (cp<int32_t>)d.gm_fs;
    const gp<const float> nrm_g = gmem(static_cast<const float *>(d.nrm));
    const gp<const uint8_t> inf = gmem(d.inf);
    const gp<float2> bkeep = gmem(static_cast<float2 *>(d.Msrt));
    const gp<const float2> S = gmem(static_cast<const float2 *>(d.S));

    // owned rows: slot (k, r) is user 16 (w + T k) + 4 g + r in VR-start order;
    // r and the last product in registers, q and the row scales in LDS
    auto blk = [&](int k) { return w + T * k; };
    auto row = [&](int k, int r) { return 16 * blk(k) + 4 * g + r; };
    // this lane's entries of the per-row LDS arrays, slot (0, 0); slot
    // (k, r) lies 16 T k + r rows further, a constant, so every access is
    // one base register plus an immediate offset
    auto ro = [](int k, int r) { return 16 * T * k + r; };
    const int r00 = 16 * w + 4 * g;
    float2 *const Qr = L.Q + r00 * 16 + j;
    float2 *const PVr = L.PV + r00 * 16 + j;
    const float *const fvr = L.fv + r00;
    const float *const ffr = L.ff + r00;
    float2 rr[BPW][4], pp[BPW][4];
    for (int ku = tid; ku < kpad; ku += T * 64) {
        float fv = 0.f, ff = 0.f;
        if (ku < K) {
            const int u = perm[ku];
            const float inv = 1.f / nrm_g[u];
            if (oahk && inf[u]) ff = inv;
            else fv = inv;
        }
        L.fv[ku] = fv;
        if (oahk) L.ff[ku] = ff;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) L.Q[ku * 16 + jj] = float2{0.f, 0.f};
    }
    if (oahk) {
        for (int i = tid; i < kpad / 4; i += T * 64) L.fslot[i] = VRK_WAVE_FCHUNKS;
        if (tid < 64) L.PF[VRK_WAVE_FCHUNKS * 64 + tid] = float2{0.f, 0.f};
        __syncthreads();
        for (int t = tid; t < d.nfch; t += T * 64) L.fslot[gmem(d.fch)[t]] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BPW; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) rr[k][r] = pp[k][r] = float2{0.f, 0.f};

    // right-hand side: s (forward) or b = H g (adjoint, from the residual
    // tiles: 16 users x antennas 16 ab + 4 kk + m at lane i + 16 kk, times the
    // rows of g; the product's output layout is the state layout). The
    // tile's 16 rows of g go through LDS (the PV buffer, free until the
    // first publish) a batch of antenna blocks at a time: every wave's blocks
    // read them from there, so each row of g leaves memory once per tile
    // instead of once per block whose band covers it. The batch is stored
    // row by row (as read from memory), antenna n of row jr at
    // span jr + (n ^ f(jr)) with f(jr) = (jr & 3) + 8 (jr >> 2): the stores
    // are contiguous runs, and the operand reads (row j, antennas
    // 4 kk + m + 16 c of the 32 lanes of a half-wave) fall in distinct banks
    if (a.adjoint) {
        const gp<const float2> HA = gmem(static_cast<const float2 *>(d.HA));
        const gp<const float2> GX = gmem(static_cast<const float2 *>(d.GX));
        // antenna blocks per batch (PV holds 16 rows x 16 nub entries), even
        // when it can be so that a row spans whole 32-entry swizzle groups
        const int nbat = nub >= 2 ? (nub & ~1) : 1;
        const int span = 16 * nbat;
        const bool swz = (span & 31) == 0;
        auto fsw = [&](int jr) { return swz ? (jr & 3) + 8 * (jr >> 2) : 0; };
        C3 acc[BPW];
#pragma unroll
        for (int k = 0; k < BPW; ++k) acc[k] = c3_zero();
        // this thread's entries e = tid + q T 64 of a batch (16 rows x span
        // antennas, at most 4 BPW per thread), loaded one batch ahead
        constexpr int kE = 4 * BPW;
        float2 gv[kE];
        auto load_batch = [&](int ab0) {
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                const int e = tid + q * T * 64;
                const int jr = e / span, n = 16 * ab0 + (e - jr * span), br = b0 + jr;
                gv[q] = float2{0.f, 0.f};
                if (e < 16 * span && br < nrhs && n < N) gv[q] = GX[(int64_t)br * d.ldgx + n];
            }
        };
        load_batch(0);
        const int fj = fsw(j);
#pragma unroll 1
        for (int ab0 = 0; ab0 < nab; ab0 += nbat) {
            __syncthreads();   // the previous batch is consumed
#pragma unroll
            for (int q = 0; q < kE; ++q) {
                const int e = tid + q * T * 64;
                if (e < 16 * span) {
                    const int jr = e / span, no = e - jr * span;
                    L.PV[jr * span + (no ^ fsw(jr))] = gv[q];
                }
            }
            __syncthreads();
            if (ab0 + nbat < nab) load_batch(ab0 + nbat);   // in flight during the products
#pragma unroll
            for (int k = 0; k < BPW; ++k) {
                const int mb = blk(k);
                if (mb >= nub) continue;
                const int lo = gmem(d.rab_lo)[mb], hi = gmem(d.rab_hi)[mb];
                const int64_t hb = gmem(d.ha_off)[mb];
                const int a0 = lo > ab0 ? lo : ab0, a1 = hi < ab0 + nbat ? hi : ab0 + nbat;
#pragma unroll 1
                for (int ab = a0; ab < a1; ab += 2) {
                    float2 h[2][4], x[2][4];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const gp<const float2> hp = HA + (hb + 4 * (int64_t)(ab + t - lo)) * 64 + lane;
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            h[t][m] = x[t][m] = float2{0.f, 0.f};
                            if (ab + t < a1) {
                                h[t][m] = hp[64 * m];
                                x[t][m] = L.PV[j * span + ((16 * (ab + t - ab0) + 4 * g + m) ^ fj)];
                            }
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int m = 0; m < 4; ++m) c3mfma(acc[k], h[t][m], x[t][m]);
                }
            }
        }
        __syncthreads();   // PV is free again for the first publish
#pragma unroll
        for (int k = 0; k < BPW; ++k) {
            const int mb = blk(k);
            if (mb >= nub) continue;
            f4 re, im;
            c3_get(acc[k], re, im);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rr[k][r] = float2{re[r], im[r]};
                if (colok) bkeep[(int64_t)b * kpad + 16 * mb + 4 * g + r] = rr[k][r];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < BPW; ++k)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ku = 16 * blk(k) + 4 * g + r;
                if (colok && blk(k) < nub && ku < K) rr[k][r] = S[(int64_t)b * d.lds + perm[ku]];
            }
    }
    // s (or b) of slot (k, r) again at the confirm pass; gq is this lane's
    // g made opaque to the compiler there, so that the addresses are formed
    // anew rather than kept live (spilled) from the first read
    auto rhs = [&](int k, int r, int gq) -> float2 {
        const int ku = 16 * blk(k) + 4 * gq + r;
        const int bq = b0 + (lane & 15);
        if (!colok || blk(k) >= nub) return float2{0.f, 0.f};
        if (a.adjoint) return bkeep[(int64_t)bq * kpad + ku];
        if (ku >= K) return float2{0.f, 0.f};
        return S[(int64_t)bq * d.lds + perm[ku]];
    };

    // Publish what the next step's products read, with the partial sums:
    // VR-OAHK writes phi_F = r / ||a||^2 on the rows of F into the chunks of
    // PF (the owners of a chunk write all four of its rows); AHK writes phi
    // to PV and adds phi^H r. Both add ||r||^2.
    auto publish = [&](float (&part)[2]) {
        part[0] = part[1] = 0.f;
#pragma unroll
        for (int k = 0; k < BPW; ++k) {
            const int mb = blk(k);
            if (mb >= nub) continue;
            // chunk 4 mb + g holds this lane's four rows; chunks without a
            // user of F write nothing (their operand is the zero spare slot)
            const int slot = oahk ? L.fslot[4 * mb + g] : 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float2 x = rr[k][r];
                const float n2 = x.x * x.x + x.y * x.y;
                part[0] += n2;
                if (oahk) {
                    const float f = ffr[ro(k, r)];
                    if (slot < VRK_WAVE_FCHUNKS) L.PF[slot * 64 + r * 16 + j] = float2{x.x * f, x.y * f};
                } else {
                    const float f = fvr[ro(k, r)];
                    PVr[ro(k, r) * 16] = float2{x.x * f, x.y * f};
                    part[1] += n2 * f;
                }
            }
        }
    };

    float sums[2];
    publish(sums);
    colsum<T, 2>(sums, L.red, 0);
    float r2 = sums[0], num = sums[1];
    const float fro2 = *gmem(static_cast<const float *>(d.fro2));
    // state of column j, identical in every lane of the column and every wave
    const float sn = sqrtf(r2);
    bool act = false;
    int fl = 0, its = 0;
    float rel = 0.f;
    if (colok) {
        if (!isfinite(sn) || !isfinite(fro2)) fl = VRK_FLAG_NONFINITE;
        else if (r2 == 0.f) fl = VRK_FLAG_CONVERGED;
        else act = true;
    }

    int64_t t_it = 0;
    for (;;) {
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
            if (__ballot(act) == 0) break;   // the same in every wave of the tile

            if constexpr (oahk) {
                // orthogonal half-step on F (gamma = 1, Prop. 1): q_F += phi_F,
                // r -= M phi_F over the chunks of F users; then phi of V to PV
                float nv[1] = {0.f};
#pragma unroll
                for (int k = 0; k < BPW; ++k) {
                    const int mb = blk(k);
                    if (mb >= nub) continue;
                    const int e0 = __builtin_amdgcn_readfirstlane(gmoff[mb]);
                    const int nf = __builtin_amdgcn_readfirstlane(gmnf[mb]);
                    f4 pr, pi;
                    block_product(GM, gmfs, e0, e0 + nf, L.PF, pr, pi);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float ff = act ? ffr[ro(k, r)] : 0.f;
                        if (ff != 0.f) {
                            const float2 q = Qr[ro(k, r) * 16];
                            Qr[ro(k, r) * 16] = float2{q.x + rr[k][r].x * ff, q.y + rr[k][r].y * ff};
                        }
                        if (act) rr[k][r] = float2{rr[k][r].x - pr[r], rr[k][r].y - pi[r]};
                        const float f = fvr[ro(k, r)];
                        const float2 x = rr[k][r];
                        PVr[ro(k, r) * 16] = float2{x.x * f, x.y * f};
                        nv[0] += (x.x * x.x + x.y * x.y) * f;
                    }
                }
                colsum<T, 1>(nv, L.red, 1);
                num = nv[0];
            }
            // aggregated step: P = M phi over every chunk of the owned blocks,
            // gamma = phi^H r / phi^H M phi
            float dn[1] = {0.f};
#pragma unroll
            for (int k = 0; k < BPW; ++k) {
                const int mb = blk(k);
                if (mb >= nub) continue;
                const int e0 = __builtin_amdgcn_readfirstlane(gmoff[mb]);
                const int e1 = __builtin_amdgcn_readfirstlane(gmoff[mb + 1]);
                f4 pr, pi;
                block_product(GM, gmc, e0, list_real_end(gmc, e0, e1), L.PV, pr, pi);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    pp[k][r] = float2{pr[r], pi[r]};
                    dn[0] += (rr[k][r].x * pr[r] + rr[k][r].y * pi[r]) * fvr[ro(k, r)];
                }
            }
            colsum<T, 1>(dn, L.red, 2);
            const float gm = (act && num > 0.f && dn[0] > 0.f) ? num / dn[0] : 0.f;
            if (gm != 0.f) {
#pragma unroll
                for (int k = 0; k < BPW; ++k) {
                    if (blk(k) >= nub) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float f = gm * fvr[ro(k, r)];
                        const float2 q = Qr[ro(k, r) * 16];
                        Qr[ro(k, r) * 16] = float2{q.x + f * rr[k][r].x, q.y + f * rr[k][r].y};
                        rr[k][r] = float2{rr[k][r].x - gm * pp[k][r].x, rr[k][r].y - gm * pp[k][r].y};
                    }
                }
            }
            publish(sums);
            colsum<T, 2>(sums, L.red, 0);
            r2 = sums[0];
            num = sums[1];
            ++t_it;
        }

        // every column stopped: x = H^H q into the output rows, and the fresh
        // residual s - M q decides (q from LDS as the products' operand)
        __syncthreads();
        if (!a.adjoint) {
            const gp<const float2> HG = gmem(static_cast<const float2 *>(d.HG));
            const cp<int32_t> agoff = (cp<int32_t>)d.ag_off, aguc = (cp<int32_t>)d.ag_uc;
            const gp<float2> row = gmem(static_cast<float2 *>(d.X)) + (int64_t)(colok ? b : 0) * d.ldx;
#pragma unroll 1
            for (int ab = w; ab < nab; ab += T) {
                // four chunks' loads in flight together, no prefetch across
                // groups (x is formed once per solve; fewer live registers)
                C3 acc = c3_zero();
                const int e0 = __builtin_amdgcn_readfirstlane(agoff[ab]);
                const int e1 = __builtin_amdgcn_readfirstlane(agoff[ab + 1]);
                int e = e0;
#pragma unroll 1
                for (; e + 3 < e1; e += 4) {
                    float2 h[4], f[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        h[i] = HG[(int64_t)(e + i) * 64 + lane];
                        f[i] = L.Q[__builtin_amdgcn_readfirstlane(aguc[e + i]) * 64 + lane];
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) c3mfma(acc, h[i], f[i]);
                }
#pragma unroll 1
                for (; e < e1; ++e)
                    c3mfma(acc, HG[(int64_t)e * 64 + lane], L.Q[__builtin_amdgcn_readfirstlane(aguc[e]) * 64 + lane]);
                f4 xr, xi;
                c3_get(acc, xr, xi);
                const int n0 = 16 * ab + 4 * g;
                // Streaming stores that fill whole 32-byte sectors: lanes g
                // and g ^ 1 of a column trade halves (row-swap move), so that
                // one store writes bytes [0, 32) and [64, 96) of the 16
                // antennas' 128-byte run and the other [32, 64) and [96, 128).
                // x is not read again here; it should not push the channel's
                // tiles out of L2.
                const f4 h0 = {xr[0], xi[0], xr[1], xi[1]}, h1 = {xr[2], xi[2], xr[3], xi[3]};
                f4 sa, sb;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(h0[c]), __float_as_uint(h1[c]),
                                                                    false, false);
                    sa[c] = __uint_as_float(p[0]);
                    sb[c] = __uint_as_float(p[1]);
                }
                if (colok) {
                    const int nb = 16 * ab;
                    if (nb + 15 < N && ((reinterpret_cast<uintptr_t>(row + nb) & 31) == 0)) {
                        const int oa = nb + 4 * (g & 2) + 2 * (g & 1), ob = oa + 4;
                        __builtin_nontemporal_store(sa, (gp<f4>)(row + oa));
                        __builtin_nontemporal_store(sb, (gp<f4>)(row + ob));
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (n0 + r < N) row[n0 + r] = float2{xr[r], xi[r]};
                    }
                }
            }
        }
        float t2[1] = {0.f};
        int gq = g;
        asm volatile("" : "+v"(gq));
#pragma unroll
        for (int k = 0; k < BPW; ++k) {
            const int mb = blk(k);
            if (mb >= nub) continue;
            const int e0 = __builtin_amdgcn_readfirstlane(gmoff[mb]);
            const int e1 = __builtin_amdgcn_readfirstlane(gmoff[mb + 1]);
            f4 pr, pi;
            block_product(GM, gmc, e0, list_real_end(gmc, e0, e1), L.Q, pr, pi);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float2 s0 = rhs(k, r, gq);
                rr[k][r] = float2{s0.x - pr[r], s0.y - pi[r]};
                t2[0] += rr[k][r].x * rr[k][r].x + rr[k][r].y * rr[k][r].y;
            }
        }
        colsum<T, 1>(t2, L.red, 1);
        // columns stopped by the rule or the iteration cap take the fresh
        // residual's verdict; a column it rejects resumes while the cap allows
        if (fl == kPending || fl == VRK_FLAG_MAXITER) {
            rel = sqrtf(t2[0]) / sn;
            if (!isfinite(rel)) fl = VRK_FLAG_NONFINITE;
            else if (rel <= (float)a.tol) fl = VRK_FLAG_CONVERGED;
            else if (t_it < a.max_iters) { fl = 0; act = true; }
            else fl = VRK_FLAG_MAXITER;
        }
        if (__ballot(act) == 0) break;
        // resume from the fresh residual (PV and PF are free after the barrier)
        publish(sums);
        colsum<T, 2>(sums, L.red, 0);
        r2 = sums[0];
        num = sums[1];
    }

    // outputs: v (or mu) in caller order and in VR-start order
    const gp<float2> V = gmem(static_cast<float2 *>(a.adjoint ? d.GS : d.V));
    const int64_t ldv = a.adjoint ? d.ldgs : d.ldv;
    const gp<float2> VS = gmem(static_cast<float2 *>(a.adjoint ? d.Msrt : d.Vsrt));
    if (colok) {
#pragma unroll
        for (int k = 0; k < BPW; ++k) {
            if (blk(k) >= nub) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ku = row(k, r);
                const float2 q = Qr[ro(k, r) * 16];
                if (V && ku < K) V[(int64_t)b * ldv + perm[ku]] = q;
                if (VS) VS[(int64_t)b * kpad + ku] = q;
            }
        }
    }
    if (tid < 16 && colok) {
        const int64_t gidx = d.rhs_base + b;
        if (a.iters) gmem(a.iters)[gidx] = its;
        if (a.relres) gmem(a.relres)[gidx] = rel;
        if (a.flags) gmem(a.flags)[gidx] = fl;
    }
}

// One workgroup per work item, dealt out by xcd_item: each XCD walks its own
// contiguous run of items, so its L2 holds the tiles of few channels at a
// time.
template <int T, int BPW, int VARIANT>
__global__ void __launch_bounds__(T * 64) __attribute__((amdgpu_waves_per_eu(BPW == 4 ? 2 : 4))) k_wave_solve(VrkSolveArgs a, const VrkWork *work, int nitems)
{
    extern __shared__ __align__(16) char smem[];
    const VrkWork wk = gmem(work)[xcd_item(blockIdx.x, nitems)];
    wave_item<T, BPW, VARIANT>(a, __builtin_amdgcn_readfirstlane(wk.prob), __builtin_amdgcn_readfirstlane(wk.tile),
                               smem);
}

template <int T, int BPW, int VARIANT>
hipError_t launch_wave(const VrkSolveArgs &a, const VrkWork *work, int32_t nitems, size_t lds, hipStream_t s,
                       int mode, int *blocks_per_cu)
{
    auto kern = k_wave_solve<T, BPW, VARIANT>;
    if (mode == 1) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, T * 64, lds);
    }
    hipLaunchKernelGGL(kern, dim3(nitems), dim3(T * 64), lds, s, a, work, nitems);
    return hipGetLastError();
}

template <int T, int BPW>
hipError_t launch_wave_variant(const VrkSolveArgs &a, const VrkWork *work, int32_t nitems, size_t lds, hipStream_t s,
                               int mode, int *bpc)
{
    if (a.variant == 1) return launch_wave<T, BPW, 1>(a, work, nitems, lds, s, mode, bpc);
    if (a.variant == 3) return launch_wave<T, BPW, 3>(a, work, nitems, lds, s, mode, bpc);
    return hipErrorInvalidValue;
}

}  // namespace

int vrk_wave_supported(int32_t variant, int32_t kpad, int32_t waves, int32_t bpw)
{
    if (variant != 1 && variant != 3) return 0;
    if (!((bpw == 4 && (waves == 1 || waves == 2 || waves == 4)) ||
          (bpw == 2 && (waves == 1 || waves == 2 || waves == 4 || waves == 8))))
        return 0;
    return kpad <= VRK_UB * waves * bpw ? 1 : 0;
}

size_t vrk_wave_lds_bytes(int32_t variant, int32_t kpad, int32_t waves)
{
    return wave_lds_layout(kpad, waves, variant == 3, nullptr, nullptr);
}

hipError_t vrk_launch_wave_solve(const VrkSolveArgs &a, const VrkWork *work, int32_t nitems, int32_t waves, int32_t bpw,
                                 size_t lds, hipStream_t s, int mode, int *bpc)
{
    if (nitems <= 0) return hipSuccess;
    if (bpw == 4) {
        if (waves == 1) return launch_wave_variant<1, 4>(a, work, nitems, lds, s, mode, bpc);
        if (waves == 2) return launch_wave_variant<2, 4>(a, work, nitems, lds, s, mode, bpc);
        if (waves == 4) return launch_wave_variant<4, 4>(a, work, nitems, lds, s, mode, bpc);
    } else if (bpw == 2) {
        if (waves == 1) return launch_wave_variant<1, 2>(a, work, nitems, lds, s, mode, bpc);
        if (waves == 2) return launch_wave_variant<2, 2>(a, work, nitems, lds, s, mode, bpc);
        if (waves == 4) return launch_wave_variant<4, 2>(a, work, nitems, lds, s, mode, bpc);
        if (waves == 8) return launch_wave_variant<8, 2>(a, work, nitems, lds, s, mode, bpc);
    }
    return hipErrorInvalidValue;
}
