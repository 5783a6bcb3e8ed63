// Vector engine, small-channel form (Nt <= 1024, K <= 64 and the channel,
// zero-padded to 16-row blocks of whole waves of 64-antenna slots, within
// 128 KiB of LDS): one workgroup of T <= 4 waves per right-hand side,
// complex64 or complex128, the same steps in the same order as the general
// form (Alg. 1 initialisation; the residual, selection and single-row
// projection of GRK and VR-OGRK; the aggregated projection of AHK; the
// orthogonal half-step on F and the aggregated step on V of VR-OAHK,
// Alg. 3).
//
// Laid out for latency. The channel sits in LDS zero-padded to whole rows of
// 64-antenna slots (and to a multiple of 16 rows), so every product is a run
// of unconditional loads and FMAs. Wave w owns NA slots (antennas
// 64 (w NA + m) + lane) and holds their x in registers; every wave holds the
// per-user state (residual, dual iterate q, row norm, VR) of user u in lane
// u, the same in all of them, and takes the same selections and step sizes
// redundantly, so the only exchanges are the residual rows (each wave's
// partial sums over its slots) and ||p||^2: one barrier each. Residual rows
// go sixteen (or four) at a time: each lane forms its partial sums of all of
// them and one reduce-scatter across the wave (six pair levels, half of the
// values to each side) totals them with about a sixth of the moves of a sum
// per row.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace {

// LDS for the zero-padded channel, in bytes.
constexpr size_t kSmallChannelBytes = 128 * 1024;

template <typename R>
using C = cx<R>;

// Pair levels of the reduce-scatter. BIT 32 and 16 pair lane l with l ^ BIT
// through the gfx950 row-swap moves (swap_sum32, swap_sum16); 8, 4, 2 and 1
// pair lanes inside a row of 16 with DPP moves (rotate by 8, mirror within
// 8, quad swaps), partners that differ in that bit. Each level leaves, in
// every lane, own + partner of one of two values a, b: a where the lane's
// bit is clear, b where set.
template <int BIT>
constexpr int pair_ctrl()
{
    return BIT == 8 ? 0x128 : BIT == 4 ? 0x141 : BIT == 2 ? 0x4E : 0xB1;
}

template <int BIT, typename R>
__device__ __forceinline__ R half_sum(R a, R b, int lane)
{
    if constexpr (BIT == 32) {
        return swap_sum32(a, b);
    } else if constexpr (BIT == 16) {
        return swap_sum16(a, b);
    } else {
        const bool hi = (lane & BIT) != 0;
        const R send = hi ? a : b, keep = hi ? b : a;   // the partner keeps the other value
        return keep + dpp_move<pair_ctrl<BIT>()>(send);
    }
}

template <int BIT, typename R>
__device__ __forceinline__ R pair_sum(R v)
{
    if constexpr (BIT == 32) return swap_sum32(v, v);
    else if constexpr (BIT == 16) return swap_sum16(v, v);
    else return v + dpp_move<pair_ctrl<BIT>()>(v);
}

template <int BIT, int H, typename R>
__device__ __forceinline__ void halve(R *v, int lane)
{
#pragma unroll
    for (int i = 0; i < H; ++i) v[i] = half_sum<BIT>(v[i], v[H + i], lane);
}

// Totals over the 64 lanes of NV values per lane (NV a power of two <= 64):
// returns in lane l the total of value l >> (6 - log2 NV). v is overwritten.
template <int NV, typename R>
__device__ __forceinline__ R reduce_scatter(R *v, int lane)
{
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV: power of two <= 64");
    if constexpr (NV >= 2) halve<32, NV / 2>(v, lane);
    if constexpr (NV >= 4) halve<16, NV / 4>(v, lane);
    if constexpr (NV >= 8) halve<8, NV / 8>(v, lane);
    if constexpr (NV >= 16) halve<4, NV / 16>(v, lane);
    if constexpr (NV >= 32) halve<2, NV / 32>(v, lane);
    if constexpr (NV >= 64) halve<1, NV / 64>(v, lane);
    R s = v[0];
    if constexpr (NV < 2) s = pair_sum<32>(s);
    if constexpr (NV < 4) s = pair_sum<16>(s);
    if constexpr (NV < 8) s = pair_sum<8>(s);
    if constexpr (NV < 16) s = pair_sum<4>(s);
    if constexpr (NV < 32) s = pair_sum<2>(s);
    if constexpr (NV < 64) s = pair_sum<1>(s);
    return s;
}

// LDS exchange slots per wave and buffer: 2 values (Re, Im) for each of up
// to 64 residual rows.
constexpr int kXch = 128;

// Per-thread view of the state a step needs.
template <typename R, int T, int NA>
struct Ctx {
    const C<R> *hd;   // the channel, zero-padded: H[u, n] at hd[u npad + n]
    int npad;
    C<R> *ph;         // this wave's broadcast slots (K)
    R *xch;           // exchange buffers [2][T][kXch]
    int w, lane, K, nx;   // wave, lane, users, exchanges so far
    int n0;           // first antenna of slot 0 of this wave, plus lane
    R xi;
    C<R> x[NA];       // x on antennas n0 + 64 m
    C<R> s, r, q;     // user `lane`
};

// Pops up to NR set bits of m (ascending) into rows; -1 past the last.
template <int NR>
__device__ __forceinline__ void pop_rows(uint64_t &m, int (&rows)[NR])
{
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        if (m) {
            rows[t] = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
        } else {
            rows[t] = -1;
        }
    }
}

// Partial sums of rows (wave-uniform, -1: none) over this wave's slots,
// totalled across the wave: on return, value j (2 t: Re of row t, 2 t + 1:
// Im) of this wave's total sits in lanes [j W, (j + 1) W), W = 32 / NR.
template <typename R, int T, int NA, int NR>
__device__ __forceinline__ R row_partials(const Ctx<R, T, NA> &c, const int (&rows)[NR])
{
    R v[2 * NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        const C<R> *h = c.hd + (int64_t)(rows[t] < 0 ? 0 : rows[t]) * c.npad + c.n0;
        R ar = 0, ai = 0;
#pragma unroll
        for (int m = 0; m < NA; ++m) {
            // explicit FMAs: the same rounding wherever this is inlined, so
            // that a row's residual does not depend on the rows beside it
            const C<R> hv = h[64 * m];
            ar = fma(hv.re, c.x[m].re, ar);
            ar = fma(-hv.im, c.x[m].im, ar);
            ai = fma(hv.re, c.x[m].im, ai);
            ai = fma(hv.im, c.x[m].re, ai);
        }
        if (rows[t] < 0) ar = ai = 0;
        v[2 * t] = ar;
        v[2 * t + 1] = ai;
    }
    return reduce_scatter<2 * NR>(v, c.lane);
}

// r_i = s_i - H[i, :] x - xi q_i for the users in m (wave-uniform mask; at
// most 64): every wave forms its partial sums, chunk after chunk; with
// several waves the partials meet in LDS (one barrier) and each lane adds
// its user's in wave order, so that every wave holds the same residual.
template <typename R, int T, int NA>
__device__ __forceinline__ void residual_set(Ctx<R, T, NA> &c, uint64_t m)
{
    int mypos = -1;   // this lane's user: index of its Re value among the exchanged values
    int base = 0;     // values exchanged so far
    R mine_re = 0, mine_im = 0;
    R *xb = c.xch + (size_t)(c.nx & 1) * T * kXch + (size_t)c.w * kXch;
    while (m) {
        if (__popcll(m) > 4) {
            int rows[16];
            pop_rows(m, rows);
            const R tot = row_partials<R, T, NA, 16>(c, rows);
            int me = -1;
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (rows[t] == c.lane) me = t;
            if constexpr (T == 1) {
                const int src = me < 0 ? 0 : 4 * me;
                const R re = __shfl(tot, src, 64), im = __shfl(tot, src + 2, 64);
                if (me >= 0) { mine_re = re; mine_im = im; mypos = 0; }
            } else {
                if ((c.lane & 1) == 0) xb[base + (c.lane >> 1)] = tot;
                if (me >= 0) mypos = base + 2 * me;
            }
            base += 32;
        } else {
            int rows[4];
            pop_rows(m, rows);
            const R tot = row_partials<R, T, NA, 4>(c, rows);
            int me = -1;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (rows[t] == c.lane) me = t;
            if constexpr (T == 1) {
                const int src = me < 0 ? 0 : 16 * me;
                const R re = __shfl(tot, src, 64), im = __shfl(tot, src + 8, 64);
                if (me >= 0) { mine_re = re; mine_im = im; mypos = 0; }
            } else {
                if ((c.lane & 7) == 0) xb[base + (c.lane >> 3)] = tot;
                if (me >= 0) mypos = base + 2 * me;
            }
            base += 8;
        }
    }
    if constexpr (T > 1) {
        __syncthreads();
        const R *xr = c.xch + (size_t)(c.nx & 1) * T * kXch;
        ++c.nx;
        if (mypos >= 0) {
#pragma unroll
            for (int w = 0; w < T; ++w) {
                mine_re += xr[w * kXch + mypos];
                mine_im += xr[w * kXch + mypos + 1];
            }
        }
    }
    if (mypos >= 0) {
#pragma clang fp contract(off)
        c.r = C<R>{c.s.re - mine_re - c.xi * c.q.re, c.s.im - mine_im - c.xi * c.q.im};
    }
}

// r_i = s_i - H[i, :] x - xi q_i for every user: rows sixteen at a time
// with their offsets known at compile time (the channel's rows are padded
// with zero rows to a multiple of 16), otherwise as residual_set.
template <typename R, int T, int NA>
__device__ __forceinline__ void residual_all(Ctx<R, T, NA> &c)
{
    constexpr int kNpad = 64 * T * NA;
    R mine_re = 0, mine_im = 0;
    R *xb = c.xch + (size_t)(c.nx & 1) * T * kXch + (size_t)c.w * kXch;
    const int nch = (c.K + 15) >> 4;
    for (int ch = 0; ch < nch; ++ch) {
        const C<R> *h = c.hd + (size_t)(16 * ch) * kNpad + c.n0;
        R v[32];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            R ar = 0, ai = 0;
#pragma unroll
            for (int m = 0; m < NA; ++m) {
                const C<R> hv = h[t * kNpad + 64 * m];
                ar = fma(hv.re, c.x[m].re, ar);
                ar = fma(-hv.im, c.x[m].im, ar);
                ai = fma(hv.re, c.x[m].im, ai);
                ai = fma(hv.im, c.x[m].re, ai);
            }
            v[2 * t] = ar;
            v[2 * t + 1] = ai;
        }
        const R tot = reduce_scatter<32>(v, c.lane);
        if constexpr (T == 1) {
            const int src = 4 * (c.lane & 15);
            const R re = __shfl(tot, src, 64), im = __shfl(tot, src + 2, 64);
            if ((c.lane >> 4) == ch) { mine_re = re; mine_im = im; }
        } else {
            if ((c.lane & 1) == 0) xb[32 * ch + (c.lane >> 1)] = tot;
        }
    }
    if constexpr (T > 1) {
        __syncthreads();
        const R *xr = c.xch + (size_t)(c.nx & 1) * T * kXch;
        ++c.nx;
        if (c.lane < c.K) {
#pragma unroll
            for (int w = 0; w < T; ++w) {
                mine_re += xr[w * kXch + 2 * c.lane];
                mine_im += xr[w * kXch + 2 * c.lane + 1];
            }
        }
    }
    if (c.lane < c.K) {
#pragma clang fp contract(off)
        c.r = C<R>{c.s.re - mine_re - c.xi * c.q.re, c.s.im - mine_im - c.xi * c.q.im};
    }
}

// The sum over the waves of one wave-uniform value per wave, in wave order.
template <typename R, int T, int NA>
__device__ __forceinline__ R across_waves(Ctx<R, T, NA> &c, R v)
{
    if constexpr (T == 1) {
        return v;
    } else {
        R *xb = c.xch + (size_t)(c.nx & 1) * T * kXch;
        if (c.lane == 0) xb[c.w * kXch] = v;
        __syncthreads();
        ++c.nx;
        R t = 0;
#pragma unroll
        for (int w = 0; w < T; ++w) t += xb[w * kXch];
        return t;
    }
}

// x += g conj(H[u, :]) on this wave's antennas (u, g wave-uniform).
template <typename R, int T, int NA>
__device__ __forceinline__ void add_row(Ctx<R, T, NA> &c, int u, C<R> g)
{
    const C<R> *h = c.hd + (int64_t)u * c.npad + c.n0;
#pragma unroll
    for (int m = 0; m < NA; ++m) {
        const C<R> t = cmulc(g, h[64 * m]);
        c.x[m].re += t.re;
        c.x[m].im += t.im;
    }
}

// p = H^H f on this wave's antennas over the users in m (f_u in lane u),
// four at a time through this wave's broadcast slots, in ascending user
// order.
template <typename R, int T, int NA>
__device__ __forceinline__ void adjoint_product(const Ctx<R, T, NA> &c, C<R> f, uint64_t m, C<R> (&p)[NA])
{
    constexpr int kNpad = 64 * T * NA;
    if (c.lane < c.K) c.ph[c.lane] = f;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < NA; ++k) p[k] = C<R>{0, 0};
    while (m) {
        int us[4];
        pop_rows(m, us);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = us[j] < 0 ? us[0] : us[j];
            C<R> fu = c.ph[u];
            if (us[j] < 0) fu = C<R>{0, 0};
            const C<R> *h = c.hd + (size_t)u * kNpad + c.n0;
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                const C<R> t = cmulc(fu, h[64 * k]);
                p[k].re += t.re;
                p[k].im += t.im;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Aggregated projection (update4) over the users with in_set in their lane:
// phi_u = r_u / ||a_u||^2, p = H^H phi, gamma = sum |r_u|^2 / ||a_u||^2 /
// (||p||^2 + xi ||phi||^2), x += gamma p, q_u += gamma phi_u.
template <typename R, int T, int NA>
__device__ __forceinline__ void aggregate(Ctx<R, T, NA> &c, bool in_set, R nrm)
{
    const R inv = in_set ? (R)1 / nrm : (R)0;
    const C<R> phi = C<R>{c.r.re * inv, c.r.im * inv};
    const R num = wave_sum_dpp(cnorm2(c.r) * inv);
    const R phin = wave_sum_dpp(cnorm2(phi));
    if (!(num > 0)) return;   // zero residual on the set: no move (the same in every wave)
    C<R> p[NA];
    adjoint_product(c, phi, __ballot(in_set), p);
    R pn = 0;
#pragma unroll
    for (int m = 0; m < NA; ++m) pn += cnorm2(p[m]);
    pn = across_waves(c, wave_sum_dpp(pn));
    const R gamma = num / (pn + c.xi * phin);
#pragma unroll
    for (int m = 0; m < NA; ++m) {
        c.x[m].re += gamma * p[m].re;
        c.x[m].im += gamma * p[m].im;
    }
    if (in_set) c.q = C<R>{c.q.re + gamma * phi.re, c.q.im + gamma * phi.im};
}

template <typename R, int T, int NA>
__global__ void __launch_bounds__(64 * T) k_small_solve(VrkSolveArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int prob = blockIdx.y;
    const VrkDesc &d = a.desc[prob];
    const int b = blockIdx.x;
    if (b >= d.nrhs) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int N = d.nt, K = d.k;
    constexpr int kNpad = 64 * T * NA;   // antennas of the zero-padded rows

    // the adjoint solve forms its right-hand side b = H g itself, below
    C<R> *X, *V;
    int64_t ldx_, ldv_;
    if (a.adjoint) {
        X = reinterpret_cast<C<R> *>(d.Xadj); ldx_ = N;
        V = reinterpret_cast<C<R> *>(d.GS); ldv_ = d.ldgs;
    } else {
        X = reinterpret_cast<C<R> *>(d.X); ldx_ = d.ldx;
        V = reinterpret_cast<C<R> *>(d.V); ldv_ = d.ldv;
    }

    Ctx<R, T, NA> c;
    c.w = w;
    c.lane = lane;
    c.K = K;
    c.nx = 0;
    c.npad = kNpad;
    c.n0 = 64 * NA * w + lane;
    c.xi = (R)d.xi;
    const bool isu = lane < K;
    const int vs = isu ? d.vs[lane] : 0, ve = isu ? d.ve[lane] : 0;
    const R nrm = isu ? reinterpret_cast<const R *>(d.nrm)[lane] : (R)1;
    const R invn = (R)1 / nrm;   // the single-row step's 1 / ||a_i||^2
    const bool inF = isu && d.inf[lane] != 0;
    c.s = C<R>{0, 0};
    if (isu && !a.adjoint) c.s = reinterpret_cast<const C<R> *>(d.S)[(int64_t)b * d.lds + lane];
    const R fro2 = *reinterpret_cast<const R *>(d.fro2);

    // LDS: the channel zero-padded to kpad = 16 ceil(K / 16) rows of kNpad
    // antennas, the exchange buffers, then per wave the broadcast slots
    const int kpad = (K + 15) & ~15;
    C<R> *hd = reinterpret_cast<C<R> *>(smem);
    R *xch = reinterpret_cast<R *>(hd + (size_t)kpad * kNpad);
    C<R> *ph = reinterpret_cast<C<R> *>(xch + (T > 1 ? 2 * T * kXch : 0)) + (size_t)w * K;
    c.hd = hd;
    c.xch = xch;
    c.ph = ph;
    // stage the channel: this thread's antennas of G users per round, so
    // that their loads overlap; zero outside the VRs
    {
        constexpr int G = 16 / NA;
        const C<R> *H = reinterpret_cast<const C<R> *>(d.H);
        for (int u0 = 0; u0 < kpad; u0 += G) {
            C<R> tmp[G * NA];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int u = u0 + g < K ? u0 + g : K - 1;
                int us = __builtin_amdgcn_readlane(vs, u), ue = __builtin_amdgcn_readlane(ve, u);
                if (u0 + g >= K) us = ue = 0;   // a padding row
#pragma unroll
                for (int m = 0; m < NA; ++m) {
                    const int n = c.n0 + 64 * m;
                    tmp[g * NA + m] = C<R>{0, 0};
                    if (n >= us && n < ue) tmp[g * NA + m] = gmem(H)[(int64_t)u * d.ldh + n];
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (u0 + g < kpad) {
#pragma unroll
                    for (int m = 0; m < NA; ++m) hd[(size_t)(u0 + g) * kNpad + c.n0 + 64 * m] = tmp[g * NA + m];
                }
        }
    }
    __syncthreads();

    if (a.adjoint) {
        // b = H g from the staged channel: the residual sweep with s = 0,
        // q = 0 and g in place of x leaves r = -H g (exactly)
        const C<R> *G = reinterpret_cast<const C<R> *>(d.GX) + (int64_t)b * d.ldgx;
#pragma unroll
        for (int m = 0; m < NA; ++m) {
            const int n = c.n0 + 64 * m;
            c.x[m] = n < N ? G[n] : C<R>{0, 0};
        }
        c.q = C<R>{0, 0};
        residual_all(c);
        if (isu) c.s = C<R>{-c.r.re, -c.r.im};
    }
#pragma unroll
    for (int m = 0; m < NA; ++m) c.x[m] = C<R>{0, 0};
    c.r = c.s;   // z0 = 0: r0 = s
    c.q = C<R>{0, 0};
    const R s2 = wave_sum_dpp(cnorm2(c.s));
    const R snorm = sqrt(s2);
    // ||r||^2 above `far` cannot round to ||r|| / ||s|| <= tol (a 1e-5
    // relative margin over the few roundings of either side), so the stop
    // test needs the square root and the division only below it
    const R ts = (R)a.tol * snorm, far = ts * ts * (R)1.00001;
    const bool can_skip = far > 0 && isfinite(far);

    int32_t flags = 0;
    int64_t t = 0;
    R rel = 0;
    const int variant = a.variant;
    // the greedy draws of the next 64 iterations, one per lane
    R udraw = 0;
    if (!isfinite(snorm) || !isfinite(fro2)) {
        flags = VRK_FLAG_NONFINITE;
    } else if (s2 == 0) {
        flags = VRK_FLAG_CONVERGED;
    } else {
        for (;;) {
            if (variant != 2) residual_all(c);   // every variant but VR-OGRK recomputes all rows
            // stop rule every check_every iterations (and at the cap)
            if (a.check_every == 1 || t % a.check_every == 0 || t >= a.max_iters) {
                const R r2 = wave_sum_dpp(cnorm2(c.r));
                if (!(can_skip && r2 > far && isfinite(r2) && t < a.max_iters)) {
                    rel = sqrt(r2) / snorm;
                    if (!isfinite(rel)) { flags = VRK_FLAG_NONFINITE; break; }
                    if (rel <= (R)a.tol) { flags = VRK_FLAG_CONVERGED; break; }
                    if (t >= a.max_iters) { flags = VRK_FLAG_MAXITER; break; }
                }
            }
            if (variant == 0 || variant == 2) {
                if ((t & 63) == 0) udraw = (R)uniform24(a.seed, t + lane, b, prob);
                const R u = lane_read(udraw, (int)(t & 63));
                const int i = select_row_64<R>(K, a.select, fro2, u, cnorm2(c.r), nrm);
                // single-row projection (update): x += gamma conj(H[i, :]),
                // q_i += gamma, gamma = r_i / ||a_i||^2
                const R inv = lane_read(invn, i);
                const C<R> g = C<R>{lane_read(c.r.re, i) * inv, lane_read(c.r.im, i) * inv};
                add_row(c, i, g);
                if (lane == i) c.q = C<R>{c.q.re + g.re, c.q.im + g.im};
                if (variant == 2) {
                    // refresh only the rows of X_i, the users whose VR meets
                    // VR_i (Theorem 2)
                    const int us = __builtin_amdgcn_readlane(vs, i), ue = __builtin_amdgcn_readlane(ve, i);
                    const bool meets = lane == i || (vs > us ? vs : us) < (ve < ue ? ve : ue);
                    residual_set(c, __ballot(isu && meets));
                }
            } else if (variant == 1) {
                aggregate(c, isu, nrm);
            } else {
                // orthogonal half-step on F with gamma = 1 (Prop. 1): the VRs
                // are disjoint, so x gains each F row's term on its own
                // antennas (H^H phi_F with phi = 0 off F)
                const R invf = inF ? (R)1 / nrm : (R)0;
                const C<R> phif = C<R>{c.r.re * invf, c.r.im * invf};
                C<R> p[NA];
                adjoint_product(c, phif, __ballot(inF), p);
#pragma unroll
                for (int m = 0; m < NA; ++m) {
                    c.x[m].re += p[m].re;
                    c.x[m].im += p[m].im;
                }
                if (inF) c.q = C<R>{c.q.re + phif.re, c.q.im + phif.im};
                const uint64_t vset = __ballot(isu && !inF);
                if (vset) {
                    residual_set(c, vset);
                    aggregate(c, isu && !inF, nrm);
                }
            }
            ++t;
        }
    }
#pragma unroll
    for (int m = 0; m < NA; ++m) {
        const int n = c.n0 + 64 * m;
        if (n < N) X[(int64_t)b * ldx_ + n] = c.x[m];
    }
    if (w == 0 && V && isu) V[(int64_t)b * ldv_ + lane] = c.q;
    if (threadIdx.x == 0) {
        const int64_t g = d.rhs_base + b;
        if (a.iters) a.iters[g] = (int32_t)t;
        if (a.relres) a.relres[g] = (float)rel;
        if (a.flags) a.flags[g] = flags;
    }
}

// Waves per right-hand side and 64-antenna slots per wave for nt antennas.
// (1, 2 or 4 waves of one slot, 4 waves of two or four slots).
void small_shape(int32_t max_nt, int *T, int *NA)
{
    const int slots = (max_nt + 63) / 64;
    *T = slots <= 1 ? 1 : slots <= 2 ? 2 : 4;
    *NA = slots <= 4 ? 1 : slots <= 8 ? 2 : 4;
}

template <typename R>
const void *small_kernel(int T, int NA)
{
    if (T == 1) return reinterpret_cast<const void *>(k_small_solve<R, 1, 1>);
    if (T == 2) return reinterpret_cast<const void *>(k_small_solve<R, 2, 1>);
    if (NA == 1) return reinterpret_cast<const void *>(k_small_solve<R, 4, 1>);
    if (NA == 2) return reinterpret_cast<const void *>(k_small_solve<R, 4, 2>);
    return reinterpret_cast<const void *>(k_small_solve<R, 4, 4>);
}

template <typename R>
hipError_t launch_small(const VrkSolveArgs &a, int32_t max_nt, size_t lds, hipStream_t s)
{
    int T, NA;
    small_shape(max_nt, &T, &NA);
    const dim3 grid((unsigned)a.max_rhs, (unsigned)a.nprob), block(64 * T);
    if (T == 1) hipLaunchKernelGGL((k_small_solve<R, 1, 1>), grid, block, lds, s, a);
    else if (T == 2) hipLaunchKernelGGL((k_small_solve<R, 2, 1>), grid, block, lds, s, a);
    else if (NA == 1) hipLaunchKernelGGL((k_small_solve<R, 4, 1>), grid, block, lds, s, a);
    else if (NA == 2) hipLaunchKernelGGL((k_small_solve<R, 4, 2>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_small_solve<R, 4, 4>), grid, block, lds, s, a);
    return hipGetLastError();
}

}  // namespace

size_t vrk_small_lds_bytes(int32_t dtype, int32_t max_nt, int32_t max_k)
{
    int T, NA;
    small_shape(max_nt, &T, &NA);
    const size_t eb = dtype == 1 ? 16 : 8, rb = dtype == 1 ? 8 : 4;
    const size_t kpad = (size_t)(max_k + 15) / 16 * 16;
    return kpad * 64 * T * NA * eb + (T > 1 ? 2 * (size_t)T * kXch * rb : 0) + (size_t)T * max_k * eb;
}

int vrk_small_supported(int32_t dtype, int32_t max_nt, int32_t max_k, int32_t masked)
{
    if (max_nt < 1 || max_nt > 1024 || max_k < 1 || max_k > 64 || masked) return 0;
    int T, NA;
    small_shape(max_nt, &T, &NA);
    const size_t eb = dtype == 1 ? 16 : 8;
    const size_t kpad = (size_t)(max_k + 15) / 16 * 16;
    return kpad * 64 * T * NA * eb <= kSmallChannelBytes;
}

hipError_t vrk_prepare_small_solve(int32_t dtype, int32_t max_nt, size_t lds_bytes)
{
    int T, NA;
    small_shape(max_nt, &T, &NA);
    const void *f = dtype == 1 ? small_kernel<double>(T, NA) : small_kernel<float>(T, NA);
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t vrk_launch_small_solve(const VrkSolveArgs &a, int32_t max_nt, size_t lds_bytes, hipStream_t s)
{
    return a.dtype == 1 ? launch_small<double>(a, max_nt, lds_bytes, s) : launch_small<float>(a, max_nt, lds_bytes, s);
}
