// Vector engine: one workgroup (4 waves) per right-hand side, for
// complex64 and complex128. The whole Kaczmarz solve of one symbol vector
// runs inside one launch with x, q, r, phi in LDS; H is read from its VR
// bands in global memory (L2-resident across the workgroups of a drop), or,
// for small channels, staged in LDS with the plan tables the steps read.
//
// Also here: row norms, MFMA tile packing, and the adjoint right-hand side
// and gradient kernels.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename R>
__device__ R block_sum(R v, R *red)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_sum_dpp(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    R t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[i];
    return t;
}

// Two block sums with one pair of barriers (slots red[0..kWaves) and
// red[kWaves..2 kWaves)).
template <typename R>
__device__ void block_sum2(R &a, R &b, R *red)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    a = wave_sum_dpp(a);
    b = wave_sum_dpp(b);
    __syncthreads();
    if (lane == 0) {
        red[w] = a;
        red[kWaves + w] = b;
    }
    __syncthreads();
    R ta = 0, tb = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        ta += red[i];
        tb += red[kWaves + i];
    }
    a = ta;
    b = tb;
}

// ---------------------------------------------------------------------------
// Row norms: nrm_i = ||H[i, VR_i]||^2 + xi (the stored norms of Alg. 1), one
// wave per row, rows spread over kNormGroups workgroups per problem; then
// ||A||_F^2 = sum_i nrm_i in index order by one thread per problem.
// ---------------------------------------------------------------------------
constexpr int kNormGroups = 64;

template <typename R>
__global__ void __launch_bounds__(kThreads) k_norms(const VrkDesc *descs)
{
    const VrkDesc &d = descs[blockIdx.x];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const cx<R> *H = reinterpret_cast<const cx<R> *>(d.H);
    R *nrm = reinterpret_cast<R *>(d.nrm);
    for (int i = blockIdx.y * kWaves + w; i < d.k; i += kNormGroups * kWaves) {
        R acc = 0;
        for (int n = d.vs[i] + lane; n < d.ve[i]; n += 64) acc += cnorm2(H[(int64_t)i * d.ldh + n]);
        acc = wave_sum(acc) + (R)d.xi;
        if (lane == 0) nrm[i] = acc;
    }
    // padded users of the MFMA engine get a unit norm (their residual is 0)
    if (blockIdx.y == 0)
        for (int i = d.k + threadIdx.x; i < d.nub * VRK_UB; i += kThreads) nrm[i] = 1;
}

template <typename R>
__global__ void __launch_bounds__(64) k_fro(const VrkDesc *descs)
{
    // the sum in index order, as one thread would take it; the wave loads
    // 64 norms at a time (all in flight) and the adds read them lane by lane
    const VrkDesc &d = descs[blockIdx.x];
    const R *nrm = reinterpret_cast<const R *>(d.nrm);
    const int lane = threadIdx.x;
    R t = 0;
    for (int i0 = 0; i0 < d.k; i0 += 64) {
        const R v = i0 + lane < d.k ? nrm[i0 + lane] : (R)0;
        const int n = d.k - i0 < 64 ? d.k - i0 : 64;
        for (int l = 0; l < n; ++l) t += lane_read(v, l);
    }
    if (lane == 0) *reinterpret_cast<R *>(d.fro2) = t;
}

// ---------------------------------------------------------------------------
// MFMA tile packing (complex64). Residual tile (ub, c): lane l = i + 16 kk
// holds H[perm[16 ub + i], 16 ab + 4 kk + m] with ab = rab_lo[ub] + c / 4,
// m = c % 4, zero outside that user's VR. Aggregation tile e of antenna
// block ab: lane l = i + 16 kk holds conj(H[perm[4 uc + kk], 16 ab + i]).
// An item is the four residual tiles 4t .. 4t + 3 (one user block, one
// antenna block), or aggregation tile t; a wave packs items t of both kinds
// for kPackQ consecutive t. The Gram tiles and F columns follow in k_gram,
// k_mf.
// ---------------------------------------------------------------------------
template <int kPackQ>
__global__ void __launch_bounds__(kThreads) k_pack(const VrkDesc *descs)
{
    // each wave takes kPackQ consecutive items of both kinds, their loads in
    // flight together: the per-item chain (offset table, row index, row
    // data) is paid once for kPackQ items (4 on deep batches; 1 when there
    // are too few items to fill the device that way)
    const VrkDesc &d = descs[blockIdx.y];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t t0 = ((int64_t)blockIdx.x * kWaves + w) * kPackQ;
    const int64_t n_ha = d.ha_off[d.nub];
    const int64_t n_hg = d.ag_off[d.nab];
    const cx<float> *H = reinterpret_cast<const cx<float> *>(d.H);
    cx<float> *HA = reinterpret_cast<cx<float> *>(d.HA);
    cx<float> *HG = reinterpret_cast<cx<float> *>(d.HG);
    const int i = lane & 15, kk = lane >> 4;
    if (t0 * 4 < n_ha) {
        // item q: the four residual tiles m = 0..3 of one (user block,
        // antenna block), tiles 4 (t0 + q) + m: lane (i, kk) loads antennas
        // 16 ab + 4 kk .. + 3 of its row (contiguous) and writes one of them
        // to each tile
        int ub[kPackQ];
        wave_segments<kPackQ>(d.ha_off, d.nub, t0 * 4, 4, ub);
        int ab[kPackQ], u[kPackQ];
        bool ok[kPackQ];
#pragma unroll
        for (int q = 0; q < kPackQ; ++q) {
            ok[q] = (t0 + q) * 4 < n_ha;
            const int b = ok[q] ? ub[q] : 0;
            ab[q] = d.rab_lo[b] + (int)(((t0 + q) * 4 - d.ha_off[b]) >> 2);
            const int ku = b * VRK_UB + i;
            u[q] = ok[q] && ku < d.k ? d.perm[ku] : -1;
        }
        cx<float> v[kPackQ][4];
        int vs[kPackQ], ve[kPackQ];
#pragma unroll
        for (int q = 0; q < kPackQ; ++q) {
            vs[q] = ve[q] = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) v[q][m] = cx<float>{0.f, 0.f};
            if (u[q] >= 0) {
                // the row's entries load beside its VR bounds, then the VR selects
                const cx<float> *h = H + (int64_t)u[q] * d.ldh;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int n = ab[q] * VRK_AB + 4 * kk + m;
                    if (n < d.nt) v[q][m] = h[n];
                }
                vs[q] = d.vs[u[q]];
                ve[q] = d.ve[u[q]];
            }
        }
#pragma unroll
        for (int q = 0; q < kPackQ; ++q) {
            if (!ok[q]) continue;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int n = ab[q] * VRK_AB + 4 * kk + m;
                const cx<float> x = n < vs[q] || n >= ve[q] ? cx<float>{0.f, 0.f} : v[q][m];
                HA[((t0 + q) * 4 + m) * 64 + lane] = x;
            }
        }
    }
    if (t0 < n_hg) {
        // item q: aggregation tile t0 + q of antenna block ab, chunk uc:
        // lane (i, kk) holds conj(H[perm[4 uc + kk], 16 ab + i])
        int ab[kPackQ];
        wave_segments<kPackQ>(d.ag_off, d.nab, t0, 1, ab);   // ag_off[ab] <= t < ag_off[ab + 1]
        int u[kPackQ];
#pragma unroll
        for (int q = 0; q < kPackQ; ++q) {
            const bool ok = t0 + q < n_hg;
            const int ku = ok ? d.ag_uc[t0 + q] * 4 + kk : d.k;
            u[q] = ku < d.k ? d.perm[ku] : -1;
        }
        cx<float> h[kPackQ];
        int vs[kPackQ], ve[kPackQ];
#pragma unroll
        for (int q = 0; q < kPackQ; ++q) {
            const int n = ab[q] * VRK_AB + i;
            h[q] = cx<float>{0.f, 0.f};
            vs[q] = ve[q] = 0;
            if (u[q] >= 0) {
                if (n < d.nt) h[q] = H[(int64_t)u[q] * d.ldh + n];
                vs[q] = d.vs[u[q]];
                ve[q] = d.ve[u[q]];
            }
        }
#pragma unroll
        for (int q = 0; q < kPackQ; ++q) {
            if (t0 + q >= n_hg) continue;
            const int n = ab[q] * VRK_AB + i;
            HG[(t0 + q) * 64 + lane] = n >= vs[q] && n < ve[q] ? cx<float>{h[q].re, -h[q].im} : cx<float>{0.f, 0.f};
        }
    }
}

// Gram tiles of M = H H^H + xi I on the FP64 matrix cores. One workgroup
// takes a group of four entries t0 .. t0 + 3 of a user block's chunk list
// (the lists are padded to multiples of four, so a group never straddles two
// blocks): D[i][4 q + kk] = sum_n H[u_i, n] conj(H[v_{q,kk}, n]) for the
// block's 16 users u_i and the four chunks' 16 users v, as three real
// v_mfma_f64_16x16x4f64 products per four antennas (Gauss), over the
// antennas where the block and any of the chunks can meet, split into
// contiguous shares, one per wave (four, or eight when there are few groups
// to fill the device); entries outside a user's VR are taken as
// zero. Lane l holds the operands of user l % 16 at antenna step offset
// l / 16 (the loads of sixteen antennas in flight together, one batch
// ahead). The waves' partial sums meet in LDS and are added in wave order,
// in double, rounded once to complex64, plus xi on the diagonal; wave q
// writes tile t0 + q, whose lane i + 16 kk holds entry (i, kk).
typedef double d4 __attribute__((ext_vector_type(4)));

template <int GW>
__global__ void __launch_bounds__(GW * 64) k_gram(const VrkDesc *descs)
{
    // partial tiles, row-major with rows padded to 17 entries: the stores
    // (a row's 16 columns) and the transposed reads (one column's 16 rows)
    // both fall in distinct LDS banks
    constexpr int kRow = 17;
    __shared__ double part[GW][3][16 * kRow];
    // (problem, group) from an XCD-contiguous walk of the grid, so that the
    // groups of one user block, which read the same rows of H, share an L2
    const int item = xcd_item(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const VrkDesc &d = descs[item / gridDim.x];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t t0 = (int64_t)(item % gridDim.x) * 4;
    if (t0 >= d.gm_off[d.nub]) return;   // the whole workgroup: no barrier reached
    const int mb = wave_segment(d.gm_off, d.nub, t0);
    const cx<float> *H = reinterpret_cast<const cx<float> *>(d.H);
    // lanes 0..15: the block's users; 16..31: the four chunks' users (-1: none)
    int ru = -1, rvs = 0, rve = 0;
    if (lane < 32) {
        int ks = -1;
        if (lane < VRK_UB) {
            ks = mb * VRK_UB + lane;
        } else {
            const int uc = d.gm_c[t0 + ((lane - VRK_UB) >> 2)];
            if (uc >= 0) ks = uc * 4 + ((lane - VRK_UB) & 3);
        }
        if (ks >= 0 && ks < d.k) {
            ru = d.perm[ks];
            rvs = d.vs[ru];
            rve = d.ve[ru];
        }
    }
    int lo_b = d.nt, hi_b = 0, lo_c = d.nt, hi_c = 0;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        const int u = __builtin_amdgcn_readlane(ru, r), a = __builtin_amdgcn_readlane(rvs, r),
                  b = __builtin_amdgcn_readlane(rve, r);
        if (u < 0 || b <= a) continue;
        if (r < VRK_UB) { lo_b = min(lo_b, a); hi_b = max(hi_b, b); }
        else { lo_c = min(lo_c, a); hi_c = max(hi_c, b); }
    }
    const int lo = max(lo_b, lo_c), hi = min(hi_b, hi_c);
    // this wave's share: batches of 16 antennas split evenly over the waves
    const int nbt = hi > lo ? (hi - lo + 15) / 16 : 0, per = (nbt + GW - 1) / GW;
    const int s0 = lo + 16 * w * per, s1 = min(hi, lo + 16 * (w + 1) * per);
    // this lane's A row (block user) and B column (chunk user), and its step offset
    const int i = lane & 15, kq = lane >> 4;
    const int ua = __shfl(ru, i, 64), avs = __shfl(rvs, i, 64), ave = __shfl(rve, i, 64);
    const int ub = __shfl(ru, VRK_UB + i, 64), bvs = __shfl(rvs, VRK_UB + i, 64), bve = __shfl(rve, VRK_UB + i, 64);
    const cx<float> *ha = H + (int64_t)(ua < 0 ? 0 : ua) * d.ldh;
    const cx<float> *hb = H + (int64_t)(ub < 0 ? 0 : ub) * d.ldh;
    d4 uu = {0, 0, 0, 0}, vv = uu, ww = uu;
    auto load = [&](int n0, cx<float> (&a)[4], cx<float> (&b)[4]) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int n = n0 + 4 * st + kq;
            a[st] = b[st] = cx<float>{0.f, 0.f};
            if (ua >= 0 && n < s1 && n >= avs && n < ave) a[st] = ha[n];
            if (ub >= 0 && n < s1 && n >= bvs && n < bve) b[st] = hb[n];
        }
    };
    cx<float> a[4], b[4], an[4], bn[4];
    if (s0 < s1) load(s0, a, b);
    for (int n0 = s0; n0 < s1; n0 += 16) {
        const bool more = n0 + 16 < s1;
        if (more) load(n0 + 16, an, bn);
        __builtin_amdgcn_sched_barrier(0);   // the next loads issue before this batch's products
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            // a conj(b) with three real products (Gauss): u = ar br,
            // v = -ai bi, w = (ar + ai)(br - bi); Re = u - v, Im = w - u - v
            const double ar = a[st].re, ai = a[st].im, br = b[st].re, bi = b[st].im;
            uu = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, uu, 0, 0, 0);
            vv = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, -bi, vv, 0, 0, 0);
            ww = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, br - bi, ww, 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                a[st] = an[st];
                b[st] = bn[st];
            }
        }
    }
    // the FP64 product's lane (j, g) holds rows g + 4 r of column j
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = ((lane >> 4) + 4 * r) * kRow + (lane & 15);
        part[w][0][o] = uu[r];
        part[w][1][o] = vv[r];
        part[w][2][o] = ww[r];
    }
    __syncthreads();
    if (w >= 4) return;   // past the barrier: waves 4.. only added range shares
    // wave q writes tile t0 + q: lane l = ie + 16 kk, D row ie, column 4 q + kk
    const int ie = lane & 15, kk = lane >> 4, src = ie * kRow + 4 * w + kk;
    double su = 0.0, sv = 0.0, sw = 0.0;
#pragma unroll
    for (int x = 0; x < GW; ++x) {
        su += part[x][0][src];
        sv += part[x][1][src];
        sw += part[x][2][src];
    }
    const int64_t t = t0 + w;
    const int uc = d.gm_c[t];
    double re = su - sv, im = sw - su - sv;
    const int ku = mb * VRK_UB + ie, kv = uc * 4 + kk;
    if (uc >= 0 && ku < d.k && kv < d.k && d.perm[ku] == d.perm[kv]) re += d.xi;
    if (uc < 0) re = im = 0.0;
    reinterpret_cast<cx<float> *>(d.GM)[t * 64 + lane] = cx<float>{(float)re, (float)im};
}

// F columns of M for the VALU orthogonal half-step: entry (ku, tt) =
// M[perm[ku]][flist[tt]], copied from the Gram tiles (the same double sums,
// rounded once): tile (ku / 16, chunk pos[f] / 4) of the block pattern,
// lane ku % 16 + 16 (pos[f] % 4); zero when the chunk is not in the pattern
// (no overlap).
__global__ void __launch_bounds__(kThreads) k_mf(const VrkDesc *descs)
{
    const VrkDesc &d = descs[blockIdx.y];
    if (!d.MF) return;
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= (int64_t)d.nub * VRK_UB * d.nmf) return;
    const int ku = (int)(idx / d.nmf), tt = (int)(idx % d.nmf);
    cx<float> v = {0.f, 0.f};
    if (ku < d.k) {
        const int mb = ku / VRK_UB, pf = d.pos[d.flist[tt]], c = pf / 4;
        for (int e = d.gm_off[mb]; e < d.gm_off[mb + 1]; ++e)
            if (d.gm_c[e] == c) {
                v = reinterpret_cast<const cx<float> *>(d.GM)[(int64_t)e * 64 + (ku % VRK_UB) + 16 * (pf % 4)];
                break;
            }
    }
    reinterpret_cast<cx<float> *>(d.MF)[idx] = v;
}

// ---------------------------------------------------------------------------
// The vector-engine solve.
// ---------------------------------------------------------------------------
template <typename R>
struct VecCtx {
    const VrkDesc *d;
    const cx<R> *H;   // the channel in memory, or its VR entries staged in LDS
    int64_t ldh;      // row stride of H
    // the plan tables the iterations read, in memory or staged in LDS
    const int32_t *vs, *ve, *flist, *vlist, *gb_off, *gb_users, *xoff, *xidx;
    const uint8_t *inf;
    cx<R> *x, *p, *r, *q, *phi, *s;
    R *nrm, *pre, *red;
    R xi;
};

// r_i = s_i - H[i, VR_i] x[VR_i] - xi q_i for the rows of `list` (all rows
// when list is null): each wave takes four rows at a time, sixteen lanes per
// row along its band, and sums over those sixteen lanes with DPP moves.
template <typename R>
__device__ void residual_rows(const VecCtx<R> &c, const int32_t *list, int n)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, rg = lane >> 4, sl = lane & 15;
    for (int t0 = w * 4; t0 < n; t0 += kWaves * 4) {
        const int t = t0 + rg;
        int i = -1;
        R ar = 0, ai = 0;
        if (t < n) {
            i = list ? list[t] : t;
            const cx<R> *h = c.H + (int64_t)i * c.ldh;
            for (int nn = c.vs[i] + sl; nn < c.ve[i]; nn += 16) {
                cx<R> hv = h[nn], xv = c.x[nn];
                ar += hv.re * xv.re - hv.im * xv.im;
                ai += hv.re * xv.im + hv.im * xv.re;
            }
        }
        ar = row16_sum(ar);
        ai = row16_sum(ai);
        if (sl == 0 && i >= 0)
            c.r[i] = {c.s[i].re - ar - c.xi * c.q[i].re, c.s[i].im - ai - c.xi * c.q[i].im};
    }
}

// Antenna n of user u's interval is visible to it: always for interval VRs;
// under the subarray model when its subarray is in the user's mask. Users of
// F and of one colour class have disjoint visible sets, so concurrent
// updates that touch only visible antennas never meet.
__device__ __forceinline__ bool visible(const VrkDesc &d, bool masked, int u, int n)
{
    return !masked || ((d.vmask[u] >> (n / d.sub_len)) & 1ull);
}

// Aggregated projection (update4) over the rows with in_set(i):
// phi_i = r_i / ||a_i||^2, p = H^H phi, gamma = sum |r_i|^2/||a_i||^2 /
// (||p||^2 + xi ||phi||^2), x += gamma p, q += gamma phi.
template <typename R, typename InSet>
__device__ void aggregate(const VecCtx<R> &c, InSet in_set, int schedule)
{
    const VrkDesc &d = *c.d;
    const int tid = threadIdx.x;
    R num = 0, phin = 0;
    for (int i = tid; i < d.k; i += kThreads) {
        cx<R> f = {0, 0};
        if (in_set(i)) {
            R inv = (R)1 / c.nrm[i];
            f = {c.r[i].re * inv, c.r[i].im * inv};
            num += cnorm2(c.r[i]) * inv;
            phin += cnorm2(f);
        }
        c.phi[i] = f;
    }
    block_sum2(num, phin, c.red);
    if (!(num > 0)) return;   // zero residual on the set: no move (uniform)
    R pn = 0;
    if (schedule == VRK_SCHED_COLOUR) {
        for (int n = tid; n < d.nt; n += kThreads) c.p[n] = {0, 0};
        __syncthreads();
        const bool masked = d.masked != 0;
        for (int col = 0; col < d.ncol; ++col) {
            // users of one class have pairwise disjoint VRs: no write conflicts
            for (int e = d.col_off[col]; e < d.col_off[col + 1]; ++e) {
                int u = d.col_users[e];
                cx<R> f = c.phi[u];
                if (f.re == 0 && f.im == 0) continue;
                const cx<R> *h = c.H + (int64_t)u * c.ldh;
                for (int n = c.vs[u] + tid; n < c.ve[u]; n += kThreads) {
                    if (!visible(d, masked, u, n)) continue;
                    cx<R> t = cmulc(f, h[n]);
                    c.p[n].re += t.re;
                    c.p[n].im += t.im;
                }
            }
            __syncthreads();
        }
        for (int n = tid; n < d.nt; n += kThreads) pn += cnorm2(c.p[n]);
    } else {
        // each thread owns antennas and gathers the users covering them
        for (int n = tid; n < d.nt; n += kThreads) {
            int g = n / VRK_GATHER_BLOCK;
            // users covering this antenna, two at a time (independent loads),
            // added in list order
            R ar = 0, ai = 0;
            const int e1 = c.gb_off[g + 1];
            for (int e = c.gb_off[g]; e < e1; e += 2) {
                cx<R> t0 = {0, 0}, t1 = {0, 0};
                const int u0 = c.gb_users[e], u1 = e + 1 < e1 ? c.gb_users[e + 1] : -1;
                const cx<R> f0 = c.phi[u0];
                if ((f0.re != 0 || f0.im != 0) && n >= c.vs[u0] && n < c.ve[u0])
                    t0 = cmulc(f0, c.H[(int64_t)u0 * c.ldh + n]);
                if (u1 >= 0) {
                    const cx<R> f1 = c.phi[u1];
                    if ((f1.re != 0 || f1.im != 0) && n >= c.vs[u1] && n < c.ve[u1])
                        t1 = cmulc(f1, c.H[(int64_t)u1 * c.ldh + n]);
                }
                ar += t0.re;
                ai += t0.im;
                ar += t1.re;
                ai += t1.im;
            }
            c.p[n] = {ar, ai};
            pn += ar * ar + ai * ai;
        }
    }
    pn = block_sum(pn, c.red + 2 * kWaves);
    R gamma = num / (pn + c.xi * phin);
    for (int n = tid; n < d.nt; n += kThreads) {
        c.x[n].re += gamma * c.p[n].re;
        c.x[n].im += gamma * c.p[n].im;
    }
    for (int i = tid; i < d.k; i += kThreads)
        if (in_set(i)) {
            c.q[i].re += gamma * c.phi[i].re;
            c.q[i].im += gamma * c.phi[i].im;
        }
    __syncthreads();
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_vec_solve(VrkSolveArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int prob = blockIdx.y;
    const VrkDesc &d = a.desc[prob];
    const int b = blockIdx.x;
    if (b >= d.nrhs) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int N = d.nt, K = d.k;

    VecCtx<R> c;
    c.d = &d;
    c.H = reinterpret_cast<const cx<R> *>(d.H);
    c.xi = (R)d.xi;
    cx<R> *base = reinterpret_cast<cx<R> *>(smem);
    c.x = base;
    c.p = c.x + N;
    c.r = c.p + N;
    c.q = c.r + K;
    c.phi = c.q + K;
    c.s = c.phi + K;
    c.nrm = reinterpret_cast<R *>(c.s + K);
    c.pre = c.nrm + K;
    c.red = c.pre + K;
    c.ldh = d.ldh;
    c.vs = d.vs;
    c.ve = d.ve;
    c.flist = d.flist;
    c.vlist = d.vlist;
    c.gb_off = d.gb_off;
    c.gb_users = d.gb_users;
    c.xoff = d.xoff;
    c.xidx = d.xidx;
    c.inf = d.inf;
    if (d.stage_h) {
        // H's VR entries into LDS after the state (16-byte aligned), rows of
        // Nt (only entries inside each VR are ever read), then the plan
        // tables the iterations read, so that no step waits on memory
        uintptr_t o = reinterpret_cast<uintptr_t>(c.red + 4 * kWaves);
        cx<R> *hs = reinterpret_cast<cx<R> *>((o + 15) & ~uintptr_t(15));
        for (int u = 0; u < K; ++u)
            for (int n = d.vs[u] + tid; n < d.ve[u]; n += kThreads) hs[(int64_t)u * N + n] = c.H[(int64_t)u * d.ldh + n];
        c.H = hs;
        c.ldh = N;
        int32_t *ts = reinterpret_cast<int32_t *>(hs + (int64_t)K * N);
        auto stage = [&](const int32_t *src, int cnt) {
            for (int e = tid; e < cnt; e += kThreads) ts[e] = src[e];
            const int32_t *dst = ts;
            ts += cnt;
            return dst;
        };
        c.vs = stage(d.vs, K);
        c.ve = stage(d.ve, K);
        c.flist = stage(d.flist, d.nf);
        c.vlist = stage(d.vlist, d.nv);
        c.gb_off = stage(d.gb_off, d.ngb + 1);
        c.gb_users = stage(d.gb_users, d.gb_off[d.ngb]);
        c.xoff = stage(d.xoff, K + 1);
        c.xidx = stage(d.xidx, d.xoff[K]);
        uint8_t *ib = reinterpret_cast<uint8_t *>(ts);
        for (int e = tid; e < K; e += kThreads) ib[e] = d.inf[e];
        c.inf = ib;
        __syncthreads();
    }
    __shared__ int sh_i;
    __shared__ R sh_g[2];

    const cx<R> *S;
    cx<R> *X, *V;
    int64_t lds_, ldx_, ldv_;
    if (a.adjoint) {
        S = reinterpret_cast<const cx<R> *>(d.Sadj); lds_ = K;
        X = reinterpret_cast<cx<R> *>(d.Xadj); ldx_ = N;
        V = reinterpret_cast<cx<R> *>(d.GS); ldv_ = d.ldgs;
    } else {
        S = reinterpret_cast<const cx<R> *>(d.S); lds_ = d.lds;
        X = reinterpret_cast<cx<R> *>(d.X); ldx_ = d.ldx;
        V = reinterpret_cast<cx<R> *>(d.V); ldv_ = d.ldv;
    }
    const R *nrm_g = reinterpret_cast<const R *>(d.nrm);
    for (int n = tid; n < N; n += kThreads) c.x[n] = {0, 0};
    R s2 = 0;
    for (int i = tid; i < K; i += kThreads) {
        cx<R> sv = S[(int64_t)b * lds_ + i];
        c.s[i] = sv;
        c.r[i] = sv;   // r0 = s since z0 = 0
        c.q[i] = {0, 0};
        c.nrm[i] = nrm_g[i];
        s2 += cnorm2(sv);
    }
    s2 = block_sum(s2, c.red);
    const R fro2 = *reinterpret_cast<const R *>(d.fro2);
    const R snorm = sqrt(s2);
    int32_t flags = 0;
    int64_t t = 0;
    R rel = 0;
    const int variant = a.variant;
    if (!isfinite(snorm) || !isfinite(fro2)) {
        flags = VRK_FLAG_NONFINITE;
    } else if (s2 == 0) {
        flags = VRK_FLAG_CONVERGED;
    } else {
        for (;;) {
            if (variant != 2) {   // every variant but VR-OGRK recomputes all rows
                residual_rows(c, nullptr, K);
                __syncthreads();
            }
            // stop rule every check_every iterations (and at the cap)
            if (a.check_every == 1 || t % a.check_every == 0 || t >= a.max_iters) {
                R r2 = 0;
                for (int i = tid; i < K; i += kThreads) r2 += cnorm2(c.r[i]);
                r2 = block_sum(r2, c.red + 3 * kWaves);
                rel = sqrt(r2) / snorm;
                if (!isfinite(rel)) { flags = VRK_FLAG_NONFINITE; break; }
                if (rel <= (R)a.tol) { flags = VRK_FLAG_CONVERGED; break; }
                if (t >= a.max_iters) { flags = VRK_FLAG_MAXITER; break; }
            }
            if (variant == 0 || variant == 2) {
                if (w == 0) {
                    R u = (R)uniform24(a.seed, t, b, prob);
                    int i = select_row_wave<R>(K, a.select, fro2, u, [&](int j) -> cx<R> {
                        return {cnorm2(c.r[j]), c.nrm[j]};
                    }, c.pre);
                    if (lane == 0) {
                        sh_i = i;
                        R inv = (R)1 / c.nrm[i];
                        sh_g[0] = c.r[i].re * inv;
                        sh_g[1] = c.r[i].im * inv;
                    }
                }
                __syncthreads();
                const int i = sh_i;
                const cx<R> g = {sh_g[0], sh_g[1]};
                // single-row projection (update): x += gamma conj(H[i, VR_i]), q_i += gamma
                const cx<R> *h = c.H + (int64_t)i * c.ldh;
                for (int n = c.vs[i] + tid; n < c.ve[i]; n += kThreads) {
                    cx<R> tv = cmulc(g, h[n]);
                    c.x[n].re += tv.re;
                    c.x[n].im += tv.im;
                }
                if (tid == 0) {
                    c.q[i].re += g.re;
                    c.q[i].im += g.im;
                }
                __syncthreads();
                if (variant == 2) {   // refresh only the rows of X_i (Theorem 2)
                    residual_rows(c, c.xidx + c.xoff[i], c.xoff[i + 1] - c.xoff[i]);
                    __syncthreads();
                }
            } else if (variant == 1) {
                aggregate(c, [](int) { return true; }, a.schedule);
            } else {
                // orthogonal half-step on F with gamma = 1 (Prop. 1): the
                // VRs are disjoint, so all of F updates concurrently (under
                // the subarray model the hulls may overlap, so only the
                // visible antennas are written)
                const bool masked = d.masked != 0;
                for (int e = 0; e < d.nf; ++e) {
                    int i = c.flist[e];
                    R inv = (R)1 / c.nrm[i];
                    cx<R> f = {c.r[i].re * inv, c.r[i].im * inv};
                    const cx<R> *h = c.H + (int64_t)i * c.ldh;
                    for (int n = c.vs[i] + tid; n < c.ve[i]; n += kThreads) {
                        if (!visible(d, masked, i, n)) continue;
                        cx<R> tv = cmulc(f, h[n]);
                        c.x[n].re += tv.re;
                        c.x[n].im += tv.im;
                    }
                    if (tid == 0) {
                        c.q[i].re += f.re;
                        c.q[i].im += f.im;
                    }
                }
                __syncthreads();
                if (d.nv > 0) {
                    residual_rows(c, c.vlist, d.nv);
                    __syncthreads();
                    const uint8_t *inf = c.inf;
                    aggregate(c, [inf](int i) { return inf[i] == 0; }, a.schedule);
                }
            }
            ++t;
        }
    }
    __syncthreads();
    for (int n = tid; n < N; n += kThreads) X[(int64_t)b * ldx_ + n] = c.x[n];
    if (V)
        for (int i = tid; i < K; i += kThreads) V[(int64_t)b * ldv_ + i] = c.q[i];
    if (tid == 0) {
        int64_t g = d.rhs_base + b;
        if (a.iters) a.iters[g] = (int32_t)t;
        if (a.relres) a.relres[g] = (float)rel;
        if (a.flags) a.flags[g] = flags;
    }
}

// ---------------------------------------------------------------------------
// Adjoint right-hand side: Sadj[b, k] = sum_{n in VR_k} H[k, n] GX[b, n].
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kThreads) k_adjoint_rhs(const VrkDesc *descs)
{
    const VrkDesc &d = descs[blockIdx.y];
    const int b = blockIdx.x;
    if (b >= d.nrhs) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const cx<R> *H = reinterpret_cast<const cx<R> *>(d.H);
    const cx<R> *g = reinterpret_cast<const cx<R> *>(d.GX) + (int64_t)b * d.ldgx;
    cx<R> *out = reinterpret_cast<cx<R> *>(d.Sadj) + (int64_t)b * d.k;
    for (int i = w; i < d.k; i += kWaves) {
        R ar = 0, ai = 0;
        for (int n = d.vs[i] + lane; n < d.ve[i]; n += 64) {
            cx<R> t = cmul(H[(int64_t)i * d.ldh + n], g[n]);
            ar += t.re;
            ai += t.im;
        }
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if (lane == 0) out[i] = {ar, ai};
    }
}

// ---------------------------------------------------------------------------
// Adjoint gradients:
//   GH[k, n] = sum_b V[b,k] conj(GX[b,n] - Xadj[b,n]) - GS[b,k] conj(X[b,n])
// on the VR band of k, and gxi = -Re sum_{b,k} conj(GS[b,k]) V[b,k].
// A workgroup takes kGradUsers consecutive users and kGradAnt antennas
// (chunks slot, slot + kGradSlots, ... of its problem), so each entry of GX,
// Xadj and X is read once per user group rather than once per user. Its
// threads form kGradStreams rows of kGradAnt lanes; row t takes the
// right-hand sides b = t, t + kGradStreams, ... and the rows' partial sums
// are added in row order. Workgroup 0 of each problem also forms gxi.
// ---------------------------------------------------------------------------
constexpr int kGradUsers = 8;
constexpr int kGradSlots = 64;
constexpr int kGradAnt = 16;
constexpr int kGradStreams = kThreads / kGradAnt;

template <typename R>
__global__ void __launch_bounds__(kThreads) k_adjoint_grads(const VrkDesc *descs)
{
    __shared__ cx<R> part[kGradStreams - 1][kGradUsers][kGradAnt];
    __shared__ R red[kWaves];
    const VrkDesc &d = descs[blockIdx.y];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int st = threadIdx.x / kGradAnt, al = threadIdx.x % kGradAnt;
    const int u0 = (int)(blockIdx.x / kGradSlots) * kGradUsers, slot = (int)(blockIdx.x % kGradSlots);
    const cx<R> *V = reinterpret_cast<const cx<R> *>(d.V);
    const cx<R> *GS = reinterpret_cast<const cx<R> *>(d.GS);
    const cx<R> *GX = reinterpret_cast<const cx<R> *>(d.GX);
    const cx<R> *XA = reinterpret_cast<const cx<R> *>(d.Xadj);
    const cx<R> *X = reinterpret_cast<const cx<R> *>(d.X);
    cx<R> *GH = reinterpret_cast<cx<R> *>(d.GH);
    if (u0 < d.k) {
        const int nu = min(kGradUsers, d.k - u0);
        const int nch = (d.nt + kGradAnt - 1) / kGradAnt;
        for (int ch = slot; ch < nch; ch += kGradSlots) {
            const int c0 = ch * kGradAnt, n = c0 + al;
            bool any = false;   // some user of the group has band entries in this chunk (uniform)
            for (int e = 0; e < nu; ++e) any = any || (d.vs[u0 + e] < c0 + kGradAnt && d.ve[u0 + e] > c0);
            if (!any) continue;
            cx<R> acc[kGradUsers];
#pragma unroll
            for (int e = 0; e < kGradUsers; ++e) acc[e] = {0, 0};
            if (n < d.nt) {
                for (int b = st; b < d.nrhs; b += kGradStreams) {
                    const cx<R> gx = GX[(int64_t)b * d.ldgx + n], xa = XA[(int64_t)b * d.nt + n];
                    const cx<R> xv = X[(int64_t)b * d.ldx + n];
                    const cx<R> df = {gx.re - xa.re, gx.im - xa.im};
#pragma unroll
                    for (int e = 0; e < kGradUsers; ++e)
                        if (e < nu) {
                            const cx<R> v = V[(int64_t)b * d.ldv + u0 + e], mu = GS[(int64_t)b * d.ldgs + u0 + e];
                            const cx<R> t1 = cmulc(v, df), t2 = cmulc(mu, xv);
                            acc[e].re += t1.re - t2.re;
                            acc[e].im += t1.im - t2.im;
                        }
                }
            }
            if (st > 0)
#pragma unroll
                for (int e = 0; e < kGradUsers; ++e) part[st - 1][e][al] = acc[e];
            __syncthreads();
            if (st == 0 && n < d.nt) {
#pragma unroll
                for (int e = 0; e < kGradUsers; ++e) {
                    const int u = u0 + e;
                    if (e < nu && n >= d.vs[u] && n < d.ve[u]) {
                        cx<R> t = acc[e];
                        for (int q = 0; q < kGradStreams - 1; ++q) {
                            t.re += part[q][e][al].re;
                            t.im += part[q][e][al].im;
                        }
                        GH[(int64_t)u * d.ldgh + n] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (blockIdx.x == 0) {
        R acc = 0;
        int64_t tot = (int64_t)d.nrhs * d.k;
        for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
            int b = (int)(e / d.k), kk = (int)(e % d.k);
            cx<R> mu = GS[(int64_t)b * d.ldgs + kk], v = V[(int64_t)b * d.ldv + kk];
            acc += mu.re * v.re + mu.im * v.im;
        }
        acc = wave_sum(acc);
        if (lane == 0) red[w] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            R t = 0;
            for (int i = 0; i < kWaves; ++i) t += red[i];
            *d.gxi = -(double)t;
        }
    }
}

}  // namespace

hipError_t vrk_launch_norms(const VrkDesc *desc, int32_t nprob, int32_t dtype, hipStream_t s)
{
    const dim3 grid((unsigned)nprob, kNormGroups);
    if (dtype == 1) {
        hipLaunchKernelGGL(k_norms<double>, grid, dim3(kThreads), 0, s, desc);
        hipLaunchKernelGGL(k_fro<double>, dim3(nprob), dim3(64), 0, s, desc);
    } else {
        hipLaunchKernelGGL(k_norms<float>, grid, dim3(kThreads), 0, s, desc);
        hipLaunchKernelGGL(k_fro<float>, dim3(nprob), dim3(64), 0, s, desc);
    }
    return hipGetLastError();
}

hipError_t vrk_launch_pack(const VrkDesc *desc, int32_t nprob, int64_t max_tiles, hipStream_t s)
{
    if (max_tiles <= 0) return hipSuccess;
    if (max_tiles * nprob >= 4 * 16384) {
        const unsigned gx = (unsigned)((max_tiles + kWaves * 4 - 1) / (kWaves * 4));
        hipLaunchKernelGGL(k_pack<4>, dim3(gx, nprob), dim3(kThreads), 0, s, desc);
    } else {
        const unsigned gx = (unsigned)((max_tiles + kWaves - 1) / kWaves);
        hipLaunchKernelGGL(k_pack<1>, dim3(gx, nprob), dim3(kThreads), 0, s, desc);
    }
    // Gram tiles: one workgroup per group of four (the per-block lists are
    // padded to multiples of four); eight waves share a group's antenna range
    // when there are few groups to fill the device
    const unsigned g4 = (unsigned)((max_tiles + 3) / 4);
    if ((int64_t)g4 * nprob < 2048)
        hipLaunchKernelGGL(k_gram<8>, dim3(g4, nprob), dim3(8 * 64), 0, s, desc);
    else
        hipLaunchKernelGGL(k_gram<4>, dim3(g4, nprob), dim3(4 * 64), 0, s, desc);
    // MF entries: at most 64 * max_tiles per problem (the plan counts them in max_tiles)
    const unsigned gm = (unsigned)((max_tiles * 64 + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_mf, dim3(gm, nprob), dim3(kThreads), 0, s, desc);
    return hipGetLastError();
}

size_t vrk_vec_lds_bytes(int32_t dtype, int32_t nt, int32_t k)
{
    size_t rb = dtype == 1 ? 8 : 4;
    return (size_t)(2 * nt + 4 * k) * 2 * rb + (size_t)(2 * k) * rb + 4 * kWaves * rb + 64;
}

hipError_t vrk_prepare_vec_solve(int32_t dtype, size_t lds_bytes)
{
    const void *f = dtype == 1 ? reinterpret_cast<const void *>(k_vec_solve<double>)
                               : reinterpret_cast<const void *>(k_vec_solve<float>);
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t vrk_launch_vec_solve(const VrkSolveArgs &a, size_t lds_bytes, hipStream_t s)
{
    dim3 grid((unsigned)a.max_rhs, (unsigned)a.nprob);
    if (a.dtype == 1) hipLaunchKernelGGL(k_vec_solve<double>, grid, dim3(kThreads), lds_bytes, s, a);
    else hipLaunchKernelGGL(k_vec_solve<float>, grid, dim3(kThreads), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t vrk_launch_adjoint_rhs(const VrkDesc *desc, int32_t nprob, int32_t max_rhs, int32_t dtype,
                                  hipStream_t s)
{
    dim3 grid((unsigned)max_rhs, (unsigned)nprob);
    if (dtype == 1) hipLaunchKernelGGL(k_adjoint_rhs<double>, grid, dim3(kThreads), 0, s, desc);
    else hipLaunchKernelGGL(k_adjoint_rhs<float>, grid, dim3(kThreads), 0, s, desc);
    return hipGetLastError();
}

hipError_t vrk_launch_adjoint_grads(const VrkDesc *desc, int32_t nprob, int32_t max_k, int32_t dtype,
                                    hipStream_t s)
{
    dim3 grid((unsigned)(((max_k + kGradUsers - 1) / kGradUsers) * kGradSlots), (unsigned)nprob);
    if (dtype == 1) hipLaunchKernelGGL(k_adjoint_grads<double>, grid, dim3(kThreads), 0, s, desc);
    else hipLaunchKernelGGL(k_adjoint_grads<float>, grid, dim3(kThreads), 0, s, desc);
    return hipGetLastError();
}

namespace {

// GH = 0 on each gap (user, first antenna, length), the hidden antennas of
// the subarray model, where h = hbar * u has no free entry: blockIdx.x is
// the problem, workgroup y takes gaps y, y + gridDim.y, ...
constexpr int kGapGroups = 16;

template <typename R>
__global__ void __launch_bounds__(kThreads) k_zero_gaps(const VrkDesc *descs)
{
    const VrkDesc &d = descs[blockIdx.x];
    cx<R> *GH = reinterpret_cast<cx<R> *>(d.GH);
    for (int e = blockIdx.y; e < d.ngap; e += kGapGroups) {
        const int u = d.gaps[3 * e], a = d.gaps[3 * e + 1], len = d.gaps[3 * e + 2];
        for (int n = a + (int)threadIdx.x; n < a + len; n += kThreads) GH[(int64_t)u * d.ldgh + n] = cx<R>{0, 0};
    }
}

}  // namespace

hipError_t vrk_launch_zero_gaps(const VrkDesc *desc, int32_t nprob, int32_t dtype, hipStream_t s)
{
    const dim3 grid((unsigned)nprob, kGapGroups);
    if (dtype == 1) hipLaunchKernelGGL(k_zero_gaps<double>, grid, dim3(kThreads), 0, s, desc);
    else hipLaunchKernelGGL(k_zero_gaps<float>, grid, dim3(kThreads), 0, s, desc);
    return hipGetLastError();
}
