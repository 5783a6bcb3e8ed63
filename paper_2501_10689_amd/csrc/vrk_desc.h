// Device-side problem descriptor shared by the host plan (plan.cpp) and the
// kernels. Plain data only; every pointer is a device address inside the
// caller's buffers or the bound workspace.
#pragma once
#include <stdint.h>

// Antennas per block of the gather lists of the vector engine.
#define VRK_GATHER_BLOCK 64
// MFMA engine geometry: 16 users x 16 right-hand sides per output tile,
// 16-antenna blocks, 4-deep reduction chunks of v_mfma_f32_16x16x4f32.
#define VRK_TILE_RHS 16
#define VRK_UB 16
#define VRK_AB 16
// users per group of the cross-wave residual reduction in the MFMA engine
#define VRK_RGROUP 32
// workgroups per problem of the ||X||_F^2 partial sums of the link metrics
#define VRK_LINK_GROUPS 16

enum { VRK_FLAG_CONVERGED = 1, VRK_FLAG_NONFINITE = 2, VRK_FLAG_MAXITER = 4 };

struct VrkDesc {
    int32_t nt, k, nrhs, nf;      // antennas, users, right-hand sides, |F|
    int32_t nv, ncol, ngb, nub;   // |V|, colour classes, gather blocks, 16-user blocks
    int32_t nab, ntile, nmf, ngap;   // 16-antenna blocks, RHS tiles of 16, columns of MF (0: none),
                                     // hidden runs inside the hulls (subarray VR model)
    double xi;
    int64_t ldh, lds, ldx, ldv, ldgx, ldgh, ldgs;
    int64_t rhs_base;             // offset of this problem's RHS in the stats arrays
    const void *H;
    const void *S;
    void *X;
    void *V;
    const void *GX;
    void *GH;
    void *GS;
    double *gxi;
    void *Sadj;                   // workspace, B x K: right-hand side H g of the adjoint
    void *Xadj;                   // workspace, B x Nt: x of the adjoint solve (H^H mu); vector engine
    void *Vfwd;                   // V of the forward solve when the caller passed none
    // VR tables, original user index unless noted
    const int32_t *vs, *ve;       // VR [start, end)
    const int32_t *xoff, *xidx;   // overlap sets X_k (CSR, includes k)
    const int32_t *flist, *vlist; // F and V = complement, ascending
    const uint8_t *inf;           // F mask
    const int32_t *col_off, *col_users;  // colour classes (CSR)
    const int32_t *gb_off, *gb_users;    // users meeting each 64-antenna block (CSR)
    const int32_t *perm, *pos;    // perm[sorted] = user, pos[user] = sorted
    void *nrm;                    // real[k]: ||a_i||^2 = ||H_i||^2 + xi (written at bind)
    void *fro2;                   // real[1]: ||A||_F^2
    // MFMA engine tables (sorted user order)
    const int32_t *rab_lo, *rab_hi;  // per 16-user block: 16-antenna block range of its bands
    const int64_t *ha_off;        // per 16-user block: first residual tile
    const int32_t *ag_off, *ag_uc;   // per 16-antenna block: 4-user chunks meeting it (CSR)
    void *HA;                     // residual tiles, 64 complex64 each
    void *HG;                     // aggregation tiles (conjugated), 64 complex64 each
    const int32_t *gm_off, *gm_c; // per 16-user block: 4-user chunks with a nonzero Gram block (CSR):
                                  // chunks holding a user of F first, then the others, padded
                                  // with -1 (zero tile) to a multiple of 4
    const int32_t *gm_nf;         // per 16-user block: its chunks holding a user of F
    void *GM;                     // Gram tiles of H H^H + xi I (VR-start order), 64 complex64 each
    // MFMA engine with adjoint buffers: v of the forward solve and mu of the
    // adjoint solve again, [rhs][nub * 16] complex64 in VR-start user order
    // (zero on the padding users), for the gradient products
    void *Vsrt, *Msrt;
    // MFMA engine with adjoint buffers: the 16 x 16 blocks (ub, ub') of
    // C = sum_b v_b mu_b^H on the Gram block pattern. Blocks of row block ub
    // are [cp_off[ub], cp_off[ub + 1]), column block cp_col[p], transposed
    // block cp_tr[p]; cp_diag[ub] is block (ub, ub). Cblk holds their
    // RHS-split partials, [block][split][16 x 16] complex64 (row-major).
    const int32_t *cp_off, *cp_col, *cp_tr, *cp_diag;
    void *Cblk;
    // MFMA engine, VR-OAHK with 1..16 users in F and a nonempty V: the F
    // columns of M, MF[ku][t] = M[perm[ku]][flist[t]] complex64 (nub * 16
    // rows, rounded once from double), and fpos[t] = pos[flist[t]]
    void *MF;
    const int32_t *fpos;
    // Subarray VR model: masked = 1 when the VRs come from subarray masks
    // (then users of F or of a colour class may have overlapping hulls, and
    // only their visible antennas are disjoint); vmask[k] = the subarrays
    // user k sees, sub_len antennas each; gaps holds ngap triples (user,
    // first antenna, length) of hidden antennas inside the hulls
    int32_t masked, sub_len;
    // vector engine: stage_h = 1 when the workgroup copies H's VR entries
    // into LDS (K x Nt, row stride Nt, after its state) before iterating
    int32_t stage_h, pad3;
    const uint64_t *vmask;
    const int32_t *gaps;
    // wave-owned MFMA engine, VR-OAHK: the 4-user chunks (VR-start order)
    // holding a user of F, ascending; at most VRK_WAVE_FCHUNKS
    int32_t nfch, pad4;
    const int32_t *fch;
    // wave-owned MFMA engine, VR-OAHK: per entry of the Gram chunk lists
    // (gm_c), the chunk's slot in the compact buffer when it holds a user of
    // F, else VRK_WAVE_FCHUNKS (the spare slot, kept zero)
    const int32_t *gm_fs;
};

// Chunks of F users the wave-owned engine keeps in its compact buffer.
#define VRK_WAVE_FCHUNKS 16

// Outputs of the link metrics of one problem (device pointers): the K x K
// effective channel E (row-major, lde), the K rates and beta.
struct VrkLinkOut {
    void *E;
    int64_t lde;
    double *rate;
    double *beta;
    double noise;   // sigma^2 / rho of the rate
};

// User blocks per tile of the MFMA adjoint gradient: the blocks 4 ubg ..
// 4 ubg + 3 that meet one antenna block share its antenna operands.
#define VRK_GRAD_UG 4

// One unit of work of the MFMA engine: a problem and a tile of 16 RHS.
struct VrkWork {
    int32_t prob, tile;
};

// Work queues of the persistent MFMA launch, one per XCD: queue q owns the
// work items [base[q], base[q] + size[q]); count[q] is its claim counter,
// zeroed by a kernel before every launch. count == null: one workgroup per
// work item instead.
#define VRK_NQUEUE 8
struct VrkQueue {
    int32_t *count;
    const int32_t *base;
    const int32_t *size;
};
