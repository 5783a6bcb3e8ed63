// Device helpers shared by the HIP kernels: complex arithmetic, wave64
// reductions, Philox4x64-10, the row selection and the complex products on
// the FP32 matrix cores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vrk_desc.h"

// AMDGPU address spaces: global memory, and the read-only constant space
// whose wave-uniform loads are scalar loads into SGPRs. Pointers read from a
// descriptor are generic; casting them to global lets the compiler issue
// global (not flat) loads, which do not hold up waits on LDS traffic.
// The host pass of hipcc type-checks the same templates for x86, which has
// no such address spaces: there the qualifiers are empty.
#ifdef __HIP_DEVICE_COMPILE__
#define VRK_GLOBAL __attribute__((address_space(1)))
#define VRK_CONST __attribute__((address_space(4)))
#else
#define VRK_GLOBAL
#define VRK_CONST
#endif
template <typename T>
__device__ __forceinline__ VRK_GLOBAL T *gmem(T *p)
{
    return (VRK_GLOBAL T *)p;
}

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b)
{
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R>
__device__ __forceinline__ R cnorm2(cx<R> a)
{
    return a.re * a.re + a.im * a.im;
}

// Sum over each row of 16 lanes with DPP moves (quad swaps, half-row and
// row mirrors): every lane of the row ends with the same value, added in the
// same order. Doubles move as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename R>
__device__ __forceinline__ R row16_sum(R v)
{
    v += dpp_move<0xB1>(v);    // quad_perm [1, 0, 3, 2]: lane ^ 1
    v += dpp_move<0x4E>(v);    // quad_perm [2, 3, 0, 1]: lane ^ 2
    v += dpp_move<0x141>(v);   // row_half_mirror: the other quad of the 8
    v += dpp_move<0x140>(v);   // row_mirror: the other half of the 16
    return v;
}

template <typename R>
__device__ __forceinline__ R lane_read(R v, int lane);

template <>
__device__ __forceinline__ float lane_read(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <>
__device__ __forceinline__ int lane_read(int v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

template <>
__device__ __forceinline__ double lane_read(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// gfx950 row-swap moves (v_permlane16_swap, v_permlane32_swap) as pair
// sums: swap_sum16(a, b) leaves a + the a of lane l ^ 16 in lanes whose bit 4
// is clear and b + the b of lane l ^ 16 where it is set (swap_sum32 the same
// for bit 5), the two terms in the same order in both lanes of a pair.
// Doubles move as two 32-bit halves, both with the same lanes.
__device__ __forceinline__ float swap_sum32(float a, float b)
{
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ float swap_sum16(float a, float b)
{
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ double swap_sum32(double a, double b)
{
    const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ab, (unsigned)bb, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ab >> 32), (unsigned)(bb >> 32), false, false);
    const double x0 = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    const double x1 = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
    return x0 + x1;
}
__device__ __forceinline__ double swap_sum16(double a, double b)
{
    const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ab, (unsigned)bb, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ab >> 32), (unsigned)(bb >> 32), false, false);
    const double x0 = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    const double x1 = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
    return x0 + x1;
}

// Sum over the 64 lanes, in every lane: the sixteen-lane row sums, then
// rows 0 + 1 and 2 + 3, then the two halves; the same order in all lanes.
template <typename R>
__device__ __forceinline__ R wave_sum_dpp(R v)
{
    v = row16_sum(v);
    return swap_sum32(swap_sum16(v, v), swap_sum16(v, v));
}

// Largest of v over lanes l and l ^ 16 (BIT 16) or l ^ 32 (BIT 32), through
// the row-swap moves of v with itself.
template <int BIT>
__device__ __forceinline__ float swap_max(float v)
{
    const auto p = BIT == 16 ? __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false)
                             : __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(p[0]), __uint_as_float(p[1]));
}
template <int BIT>
__device__ __forceinline__ double swap_max(double v)
{
    const long long b = __double_as_longlong(v);
    const auto lo = BIT == 16 ? __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false)
                              : __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = BIT == 16 ? __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false)
                              : __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return fmax(__longlong_as_double(((long long)hi[0] << 32) | lo[0]),
                __longlong_as_double(((long long)hi[1] << 32) | lo[1]));
}

// Largest value over the 64 lanes, in every lane (exact: no rounding).
template <typename R>
__device__ __forceinline__ R wave_max_dpp(R v)
{
    v = fmax(v, dpp_move<0xB1>(v));
    v = fmax(v, dpp_move<0x4E>(v));
    v = fmax(v, dpp_move<0x141>(v));
    v = fmax(v, dpp_move<0x140>(v));
    return swap_max<32>(swap_max<16>(v));
}

template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <typename R>
__device__ __forceinline__ R wave_sum(R v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <typename R>
__device__ __forceinline__ R wave_max(R v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

// DPP move with explicit row and bank masks: lanes outside the masks, and
// lanes whose source is outside their row, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_zero(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_zero(float v)
{
    return __int_as_float(dpp_zero<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_zero(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_zero<CTRL, ROWS>((int)b), hi = dpp_zero<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive prefix sum across the 64 lanes with DPP moves only: shifts by 1,
// 2, 4, 8 inside each row of 16 (Hillis-Steele), then the last lane of rows
// 0 and 2 added to rows 1 and 3 (row_bcast:15) and lane 31 to rows 2 and 3
// (row_bcast:31). The total is in lane 63.
template <typename R>
__device__ __forceinline__ R wave_scan(R v, int /*lane*/)
{
    v += dpp_zero<0x111, 0xF>(v);
    v += dpp_zero<0x112, 0xF>(v);
    v += dpp_zero<0x114, 0xF>(v);
    v += dpp_zero<0x118, 0xF>(v);
    v += dpp_zero<0x142, 0xA>(v);
    v += dpp_zero<0x143, 0xC>(v);
    return v;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x64
// S-box with the published multipliers and Weyl key increments. Returns
// the first output word.
__device__ __forceinline__ uint64_t philox4x64_10_w0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                     uint64_t c3, uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return c0;
}

// u = top 24 bits of Philox(key (seed, 0), counter (step, rhs, prob, 0)) / 2^24,
// exactly representable in float and double.
__device__ __forceinline__ double uniform24(uint64_t seed, int64_t step, int64_t rhs, int64_t prob)
{
    uint64_t w = philox4x64_10_w0((uint64_t)step, (uint64_t)rhs, (uint64_t)prob, 0, seed, 0);
    return (double)(w >> 40) * (1.0 / 16777216.0);
}

// Row selection by one wave (Sec. IV-A; Sec. III-A for the randomized
// criteria). The threshold rule keeps rows with rho_i = |r_i|^2/||a_i||^2
// >= theta, theta = min(rho_max, (rho_max + ||r||^2/||A||_F^2)/2) (the
// cited greedy randomized Kaczmarz criterion), weighted by |r_i|^2;
// RESIDUAL keeps every row, weighted by |r_i|^2; MAX returns the first
// argmax of rho; ENERGY weights row i by ||a_i||^2 and UNIFORM every row by
// 1, whatever the residual. Sampling: smallest index whose inclusive prefix
// of weights exceeds u * total, else the last index of positive weight.
//
// K <= 64 users, user i in lane i: w2 = |r_i|^2 and nrm = ||a_i||^2 of the
// lane's user (ignored on lanes >= K). Straight-line, every intermediate in
// registers.
template <typename R>
__device__ int select_row_64(int K, int rule, R fro2, R u, R w2, R nrm)
{
    const int lane = threadIdx.x & 63;
    const bool in = lane < K;
    R wt;
    int last = K - 1;
    if (rule == 3 || rule == 4) {
        // residual-free criteria
        wt = in ? (rule == 3 ? nrm : (R)1) : (R)0;
    } else {
        const R rho = in ? w2 / nrm : (R)-1;
        const R rr = wave_sum_dpp(in ? w2 : (R)0);
        // first argmax: the largest rho, then the first lane holding it
        const R best = wave_max_dpp(rho);
        const uint64_t at = __ballot(in && rho == best);
        const int bi = at ? __ffsll((unsigned long long)at) - 1 : 0;
        if (rule == 2) return bi;
        R theta = 0;
        if (rule == 0) {
            theta = (R)0.5 * (best + rr / fro2);
            if (theta > best) theta = best;
        }
        const bool keep = in && (rule == 1 || rho >= theta);
        wt = (keep && w2 > 0) ? w2 : (R)0;
        const uint64_t pos = __ballot(wt > 0);
        last = pos ? 63 - __clzll(pos) : bi;
    }
    const R v = wave_scan(wt, lane);
    const R target = u * lane_read(v, 63);
    const uint64_t hit = __ballot(in && v > target);
    return hit ? __ffsll((unsigned long long)hit) - 1 : last;
}

// The same selection for any K: get(i) returns {|r_i|^2, ||a_i||^2} for user
// i (original index order); `pre` is LDS scratch of K entries owned by the
// calling wave (unused for K <= 64).
template <typename R, typename Get>
__device__ int select_row_wave(int K, int rule, R fro2, R u, Get get, R *pre)
{
    const int lane = threadIdx.x & 63;
    if (K <= 64) {
        cx<R> wn = {0, 1};
        if (lane < K) wn = get(lane);
        return select_row_64<R>(K, rule, fro2, u, wn.re, wn.im);
    }
    if (rule == 3 || rule == 4) {
        // residual-free criteria: one prefix pass over the weights
        R carry = 0;
        for (int base = 0; base < K; base += 64) {
            const int i = base + lane;
            R wt = 0;
            if (i < K) wt = rule == 3 ? get(i).im : (R)1;
            const R v = wave_scan(wt, lane);
            if (i < K) pre[i] = carry + v;
            carry += lane_read(v, 63);
        }
        const R target = u * carry;
        __builtin_amdgcn_wave_barrier();
        for (int base = 0; base < K; base += 64) {
            const int i = base + lane;
            const uint64_t hit = __ballot(i < K && pre[i] > target);
            if (hit) return base + __ffsll((unsigned long long)hit) - 1;
        }
        return K - 1;
    }
    R rr = 0, best = -1;
    int bi = 0x7fffffff;
    for (int base = 0; base < K; base += 64) {
        int i = base + lane;
        if (i < K) {
            cx<R> wn = get(i);
            R rho = wn.re / wn.im;
            rr += wn.re;
            if (rho > best) { best = rho; bi = i; }
        }
    }
    rr = wave_sum_dpp(rr);
    // first argmax: within each 16-lane row by DPP moves, then the four row
    // winners (read as scalars) in row order; the same order in every lane
    auto take = [&](R ob, int oi) {
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    };
    take(dpp_move<0xB1>(best), dpp_move<0xB1>(bi));
    take(dpp_move<0x4E>(best), dpp_move<0x4E>(bi));
    take(dpp_move<0x141>(best), dpp_move<0x141>(bi));
    take(dpp_move<0x140>(best), dpp_move<0x140>(bi));
    {
        R rb = lane_read(best, 0);
        int ri = __builtin_amdgcn_readlane(bi, 0);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            const R ob = lane_read(best, 16 * r);
            const int oi = __builtin_amdgcn_readlane(bi, 16 * r);
            if (ob > rb || (ob == rb && oi < ri)) { rb = ob; ri = oi; }
        }
        best = rb;
        bi = ri;
    }
    if (bi >= K) bi = 0;   // unreachable for finite residuals; keeps the index in range
    if (rule == 2) return bi;
    R theta = 0;
    if (rule == 0) {
        theta = (R)0.5 * (best + rr / fro2);
        if (theta > best) theta = best;
    }
    R carry = 0;
    int last = bi;
    for (int base = 0; base < K; base += 64) {
        int i = base + lane;
        R wt = 0;
        if (i < K) {
            cx<R> wn = get(i);
            bool in = (rule == 1) || (wn.re / wn.im >= theta);
            wt = (in && wn.re > 0) ? wn.re : (R)0;
        }
        R v = wave_scan(wt, lane);
        if (i < K) pre[i] = carry + v;
        uint64_t pos = __ballot(wt > 0);
        if (pos) last = base + 63 - __clzll(pos);
        carry += lane_read(v, 63);
    }
    R target = u * carry;
    __builtin_amdgcn_wave_barrier();
    for (int base = 0; base < K; base += 64) {
        int i = base + lane;
        uint64_t hit = __ballot(i < K && pre[i] > target);
        if (hit) return base + __ffsll((unsigned long long)hit) - 1;
    }
    return last;
}

// ---------------------------------------------------------------------------
// FP32 matrix cores (v_mfma_f32_16x16x4f32). A is 16 x 4 (lane l holds row
// l % 16, reduction index l / 16), B is 4 x 16 (lane l holds reduction index
// l / 16, column l % 16), C and D are 16 x 16 (lane l holds rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16).
// ---------------------------------------------------------------------------
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

// Sum over the four lanes j, j + 16, j + 32, j + 48 of a column of the C
// layout, in every one of them: gfx950's row-swap moves (16-lane rows, then
// 32-lane halves), (v_j + v_j+16) + (v_j+32 + v_j+48) in the same order in
// all four lanes.
__device__ __forceinline__ float col4_sum(float v)
{
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// Workgroup x of a launch of n runs on XCD x % VRK_NQUEUE (the order in
// which the dispatcher deals workgroups out). This returns the work item it
// takes so that each XCD walks its own contiguous run of the items, x / 8
// ascending (split evenly when 8 does not divide n): items next to each
// other in the list share one L2 and run at about one time.
__device__ __forceinline__ int xcd_item(int x, int n)
{
    const int q = n / VRK_NQUEUE, rem = n % VRK_NQUEUE, xq = x % VRK_NQUEUE, iq = x / VRK_NQUEUE;
    return xq < rem ? xq * (q + 1) + iq : rem * (q + 1) + (xq - rem) * q + iq;
}

// Segments of Q wave-uniform positions t0 + q stride in a nondecreasing
// offset table off[0 .. n] with off[0] <= t: s[q] with off[s] <= t < off[s + 1]
// (empty segments skipped; n for a position at or past off[n]), counted as
// the entries off[1 .. n] that are <= t. Every lane loads its share of the
// table once and ballots count for all Q positions, so the search costs one
// memory latency rather than one per step. Call it with the whole wave
// active.
template <int Q, typename T>
__device__ __forceinline__ void wave_segments(const T *offp, int n, int64_t t0, int64_t stride, int (&s)[Q])
{
    const auto off = gmem(offp);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = 0;
    for (int c0 = 0; c0 < n; c0 += 256) {
        int64_t v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = 1 + c0 + 64 * c + lane;
            v[c] = j <= n ? (int64_t)off[j] : INT64_MAX;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int q = 0; q < Q; ++q) s[q] += __popcll(__ballot(v[c] <= t0 + q * stride));
    }
}

template <typename T>
__device__ __forceinline__ int wave_segment(const T *offp, int n, int64_t t)
{
    int s[1];
    wave_segments<1>(offp, n, t, 0, s);
    return s[0];
}
