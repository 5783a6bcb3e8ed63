// Host-side launchers of the HIP kernels (defined in the .hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vrk.h"
#include "vrk_desc.h"

struct VrkSolveArgs {
    const VrkDesc *desc;      // device array [nprob]
    int32_t nprob;
    int32_t max_rhs;          // largest nrhs over the problems (grid x of the vector engine)
    int32_t dtype;            // 0 complex64, 1 complex128
    int32_t variant, select, schedule;
    int32_t adjoint;          // 0: S -> X, V; 1: Sadj -> Xadj, GS
    double tol;
    int64_t max_iters;
    int64_t check_every;      // stop rule tested when the iteration count is a multiple (>= 1)
    uint64_t seed;
    int32_t *iters;
    float *relres;
    int32_t *flags;
};

// Row norms ||a_i||^2 = ||H[i, VR_i]||^2 + xi and ||A||_F^2, per problem.
hipError_t vrk_launch_norms(const VrkDesc *desc, int32_t nprob, int32_t dtype, hipStream_t s);
// MFMA residual / aggregation tiles from the VR bands of H.
hipError_t vrk_launch_pack(const VrkDesc *desc, int32_t nprob, int64_t max_tiles, hipStream_t s);

// Vector engine: one workgroup per right-hand side.
size_t vrk_vec_lds_bytes(int32_t dtype, int32_t nt, int32_t k);
hipError_t vrk_prepare_vec_solve(int32_t dtype, size_t lds_bytes);   // LDS attribute, once at bind
hipError_t vrk_launch_vec_solve(const VrkSolveArgs &a, size_t lds_bytes, hipStream_t s);

// MFMA engine: 16 right-hand sides per workgroup (complex64).
// 8 or 16 waves per tile, at most 16 users per wave (kpad: K rounded up to 16).
int vrk_mfma_supported(int32_t kpad, int32_t waves);
// (row, column) entries per thread of the solve (1, 2 or 4), 0 if unsupported.
int vrk_mfma_entries(int32_t kpad, int32_t waves);
size_t vrk_mfma_lds_bytes(int32_t kpad, int32_t nab, int32_t waves, int32_t greedy, int32_t nmf);
// mode 0 launches (grid = work items, or the persistent grid when q.count is
// set); mode 1 only sets the kernel's LDS attribute and writes its resident
// workgroups per CU to *blocks_per_cu (called once at bind, never during
// graph capture).
hipError_t vrk_launch_mfma_solve(const VrkSolveArgs &a, const VrkWork *work, const VrkQueue &q, int32_t grid,
                                 int32_t waves, int32_t ep, size_t lds_bytes, hipStream_t s, int mode,
                                 int *blocks_per_cu);

// Wave-owned MFMA engine (AHK and VR-OAHK, complex64): one workgroup of
// `waves` waves per 16-RHS tile, each wave owning up to `bpw` (4 or 2)
// 16-user row blocks; supported for waves 1, 2, 4 with bpw 4 and 1, 2, 4, 8
// with bpw 2, kpad <= 16 waves bpw. mode as vrk_launch_mfma_solve.
int vrk_wave_supported(int32_t variant, int32_t kpad, int32_t waves, int32_t bpw);
size_t vrk_wave_lds_bytes(int32_t variant, int32_t kpad, int32_t waves);
hipError_t vrk_launch_wave_solve(const VrkSolveArgs &a, const VrkWork *work, int32_t nitems, int32_t waves, int32_t bpw,
                                 size_t lds, hipStream_t s, int mode, int *blocks_per_cu);

// Adjoint pieces: b = H g (right-hand side of the adjoint solve) and the
// gradient assembly.
hipError_t vrk_launch_adjoint_rhs(const VrkDesc *desc, int32_t nprob, int32_t max_rhs,
                                  int32_t dtype, hipStream_t s);
hipError_t vrk_launch_adjoint_grads(const VrkDesc *desc, int32_t nprob, int32_t max_k,
                                    int32_t dtype, hipStream_t s);
// Subarray VR model: GH = 0 on the hidden antennas inside each hull (the
// desc's gap triples), after either engine's gradient kernels.
hipError_t vrk_launch_zero_gaps(const VrkDesc *desc, int32_t nprob, int32_t dtype, hipStream_t s);
// Link metrics after a solve with S = I_K: effective channel E = H X^T on
// each user's VR (MFMA plans: (M - xi I) V^T from the Gram tiles), beta =
// 1 / ||X||_F and the per-user rates (one table entry of outs per problem;
// dtype 0 complex64, 1 complex128; mfma: the plan is the MFMA engine's;
// part: VRK_LINK_GROUPS doubles per problem of workspace).
hipError_t vrk_launch_link(const VrkDesc *desc, const VrkLinkOut *outs, int32_t nprob, int32_t max_k, int32_t dtype,
                           int32_t mfma, double *part, hipStream_t s);
// MFMA version of the gradient assembly (complex64, plans of the MFMA
// engine, whose solve forms b = H g itself and leaves H^H mu unformed).
// GH = sum_b v_b g_b^H - (C + C^H) H with C = sum_b v_b mu_b^H and
// gxi = -Re tr C. C tiles are (problem, C block, RHS split, row block): the
// first nctiles workgroups of the first kernel write their partials to each
// problem's Cblk (csplit, 1..4, per block). Band tiles are (problem,
// user-block group, antenna block, flags: bit 0 first tile of its problem,
// bit 1 unused, bits 2.. on a problem's first tile: its problem's tile
// count). nsplit > 1 splits each band tile's RHS range over nsplit
// workgroups writing partials to gpart (ntiles * nsplit * VRK_GRAD_UG * 256
// complex64), else they write GH. A second kernel, one workgroup per run
// (first tile, tile count, flags: bit 0 first run of its problem, 0) of
// consecutive band tiles of one user-block group, sums the partials in
// fixed order, subtracts (C + C^H) H on the band and writes gxi. order
// (ntiles entries) lists the band tiles in dispatch order, by problem and
// antenna block.
hipError_t vrk_launch_adjoint_grads_mfma(const VrkDesc *desc, const int4 *tiles, const int32_t *order, int32_t ntiles,
                                         int32_t nsplit,
                                         const int4 *ctiles, int32_t nctiles, int32_t csplit, const int4 *runs,
                                         int32_t nruns, float2 *gpart, hipStream_t s);

// Vector engine, small-channel form: T <= 4 waves per right-hand side (one
// per 64-antenna slot, up to four slots each), the channel zero-padded in
// LDS, x and the per-user state in registers; for nt <= 1024, k <= 64,
// interval VRs and the padded channel (16 ceil(k / 16) rows of 64, 128, 256,
// 512 or 1024 antennas) within 128 KiB.
int vrk_small_supported(int32_t dtype, int32_t max_nt, int32_t max_k, int32_t masked);
size_t vrk_small_lds_bytes(int32_t dtype, int32_t max_nt, int32_t max_k);
hipError_t vrk_prepare_small_solve(int32_t dtype, int32_t max_nt, size_t lds_bytes);   // LDS attribute, at bind
hipError_t vrk_launch_small_solve(const VrkSolveArgs &a, int32_t max_nt, size_t lds_bytes, hipStream_t s);
