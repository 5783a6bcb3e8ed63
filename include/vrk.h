/*
 * vrk.h - C ABI of libvrk.so: VR-banded Kaczmarz RZF precoding on MI355X.
 *
 * What it computes (paper: "Low-Complexity Iterative Precoding Design for
 * Near-field Multiuser Systems With Spatial Non-Stationarity"):
 *   the RZF-precoded vector x = H^H (H H^H + xi I)^-1 s of each symbol
 *   vector s (precoding equation, Sec. II-C), as the first Nt entries of the
 *   minimum-norm solution of the consistent augmented system
 *   [H, sqrt(xi) I_K] z = s (Theorem 1, Sec. III-B), and v = (H H^H + xi I)^-1 s
 *   as its scaled last K entries (Remark 1). The system is solved by one of
 *   four Kaczmarz sweeps started from z = 0 (Alg. 1 initialisation):
 *     VRK_GRK      greedy randomized Kaczmarz (Sec. IV-A)
 *     VRK_AHK      aggregation-hyperplane Kaczmarz, eqs. (update4) and
 *                  (coefficient) (Sec. V-A)
 *     VRK_VR_OGRK  GRK refreshing only the overlapping rows X_i (Alg. 2,
 *                  Theorem 2)
 *     VRK_VR_OAHK  orthogonal-set half-step (Theorem 4, Prop. 1) then an
 *                  aggregated half-step on the rest (Alg. 3)
 *
 * Layout. H is row-major K x Nt interleaved complex (row k = the channel
 * user k sees: y_k = sum_n H[k,n] x[n]; the paper's channel matrix is its
 * conjugate transpose). User k's visibility region (VR) is the half-open
 * antenna interval [vr_start[k], vr_start[k] + vr_len[k]); only those
 * entries of H are read, the rest are taken to be zero (VR mask of the
 * channel equation). S, X, V hold one vector per row: S is B x K, X is
 * B x Nt, V is B x K. Complex64 = two float32, complex128 = two float64.
 *
 * Ownership. All device buffers belong to the caller and must outlive the
 * plan. The library never allocates device memory: the caller supplies one
 * workspace of the size vrk_plan_create reports. vrk_solve and
 * vrk_solve_adjoint only enqueue kernels on the given stream (no host
 * synchronisation, no allocation, no host<->device copy), so they can be
 * captured into a HIP graph.
 *
 * Errors. Every call returns a vrk_status; argument errors are found on
 * the host before anything is enqueued (VRK_EINVAL), and vrk_last_error()
 * gives a thread-local message. Outcomes of the iteration are per-RHS
 * flags written on the device: bit 0 converged, bit 1 non-finite input or
 * iterate, bit 2 stopped at max_iters (x is then the last iterate).
 */
#ifndef VRK_H
#define VRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VRK_OK = 0,
    VRK_EINVAL = 1,       /* bad argument (sizes, strides, VR bounds, xi, tol, null pointer) */
    VRK_EUNSUPPORTED = 2, /* valid but not supported by the chosen engine (e.g. LDS budget) */
    VRK_EWORKSPACE = 3,   /* workspace null, misaligned or smaller than reported */
    VRK_EHIP = 4,         /* a HIP runtime call failed (message in vrk_last_error) */
    VRK_ESTATE = 5        /* call order violated (solve before bind, adjoint without buffers) */
} vrk_status;

typedef enum { VRK_GRK = 0, VRK_AHK = 1, VRK_VR_OGRK = 2, VRK_VR_OAHK = 3 } vrk_variant;

/* Row selection of the single-row sweeps VRK_GRK and VRK_VR_OGRK: the greedy
 * rules of Sec. IV-A and, as the benchmarks of the simulation section, the
 * residual-free criteria of the randomized Kaczmarz method (Sec. III-A).
 *  BAIWU    threshold-and-sample rule of the greedy randomized Kaczmarz the
 *           paper cites: rows with |r_i|^2 >= eps ||r||^2 ||a_i||^2,
 *           eps = (max_i |r_i|^2/||a_i||^2 / ||r||^2 + 1/||A||_F^2) / 2, are
 *           sampled with probability proportional to |r_i|^2.
 *  RESIDUAL the printed rule p_i = |r_i|^2 / ||r||^2.
 *  MAX      argmax_i |r_i|^2 / ||a_i||^2 (lowest index on ties): greedy
 *           Kaczmarz (GK of Table I).
 *  ENERGY   p_i = ||a_i||^2 / ||A||_F^2, the energy criterion (randomized
 *           Kaczmarz; with VRK_GRK the sweep is that method).
 *  UNIFORM  p_i = 1 / K, the uniform criterion (with VRK_GRK: URK of Table I).
 * Sampling draws u = (Philox4x64-10(key (seed, 0), counter (step, rhs, prob, 0))[0]
 * >> 40) * 2^-24 and picks the smallest row index whose inclusive prefix of
 * weights exceeds u times their total. The stop rule still evaluates the
 * residual of every row. */
typedef enum {
    VRK_SEL_BAIWU = 0,
    VRK_SEL_RESIDUAL = 1,
    VRK_SEL_MAX = 2,
    VRK_SEL_ENERGY = 3,
    VRK_SEL_UNIFORM = 4
} vrk_select;

typedef enum { VRK_C64 = 0, VRK_C128 = 1 } vrk_dtype;

/* Execution engine. VECTOR: one workgroup per right-hand side, vector ALU,
 * complex64 or complex128 (a small-channel form for nt <= 1024, k <= 64:
 * see vrk_options.tile_waves). MFMA: 16 right-hand sides per workgroup sharing
 * H, residual and aggregation as FP32 matrix-core products (complex64
 * only). AUTO picks MFMA for complex64 problems with >= 16 right-hand
 * sides, VECTOR otherwise. */
typedef enum { VRK_ENGINE_AUTO = 0, VRK_ENGINE_VECTOR = 1, VRK_ENGINE_MFMA = 2 } vrk_engine;

/* Schedule of the aggregated update H^H phi in the VECTOR engine:
 * GATHER  each thread owns antennas and sums over the users covering them;
 * COLOUR  users in one colour class (pairwise disjoint VRs, Lemma 1) are
 *         scattered concurrently, classes one after another. */
typedef enum { VRK_SCHED_AUTO = 0, VRK_SCHED_GATHER = 1, VRK_SCHED_COLOUR = 2 } vrk_schedule;

/* One channel drop with its batch of symbol vectors. */
typedef struct {
    int32_t nt, k;                     /* antennas >= 1, users >= 1 (k >= nt allowed) */
    double xi;                         /* regulariser, finite and > 0 */
    const void *H;   int64_t ldh;      /* device, K x Nt, row stride ldh >= nt (elements) */
    const int32_t *vr_start;           /* HOST [k], 0 <= start */
    const int32_t *vr_len;             /* HOST [k], 0 <= len, start + len <= nt */
    int32_t nrhs;                      /* B >= 0 */
    const void *S;   int64_t lds;      /* device, B x K, lds >= k */
    void *X;         int64_t ldx;      /* device out, B x Nt, ldx >= nt */
    void *V;         int64_t ldv;      /* device out, B x K (nullable) */
    /* Adjoint buffers; all null unless vrk_solve_adjoint is used. */
    const void *GX;  int64_t ldgx;     /* device in, B x Nt: 2 dL/d conj(x) */
    void *GH;        int64_t ldgh;     /* device out, K x Nt: dL/dH on VR entries (others untouched) */
    void *GS;        int64_t ldgs;     /* device out, B x K: dL/ds */
    double *gxi;                       /* device out, one double: dL/dxi */
    /* Subarray VR model (Sec. II: the array split into S subarrays of Nt / S
     * antennas, user k seeing the subarrays of M_k). Null vr_mask: the VRs
     * are the intervals above. Otherwise vr_mask[k] has bit s set when
     * subarray s is visible to user k, [vr_start[k], vr_start[k] + vr_len[k])
     * must be the hull of those subarrays ((0, 0) for none), and H must be
     * zero on the hidden antennas inside the hull (h_k = hbar_k * u_k); the
     * kernels read H on the hull as given. Two users then overlap when their
     * masks share a subarray: that decides X_k, the Gram block pattern and
     * F, which is built by the reducing-peeling heuristic the paper cites for
     * problem max_set (degree-0 and degree-1 vertices join F, the latter
     * deleting its neighbour; otherwise the vertex of largest degree is
     * peeled; ties to the smallest index; peeled vertices then rejoin, latest
     * first, when no neighbour is in F). Colour classes come from a greedy
     * colouring of the same graph (users in VR-start order, smallest free
     * colour); concurrent updates of F or of a class write only visible
     * antennas. vrk_solve_adjoint writes GH = 0 on the hidden antennas of
     * each hull. */
    const uint64_t *vr_mask;           /* HOST [k] or null */
    int32_t n_sub;                     /* S, 1..64, nt % S == 0 (with vr_mask) */
} vrk_problem;

typedef struct {
    int32_t variant;     /* vrk_variant */
    int32_t select;      /* vrk_select (greedy variants only) */
    int32_t dtype;       /* vrk_dtype of H, S, X, V, GX, GH, GS */
    int32_t engine;      /* vrk_engine */
    double tol;          /* stop when ||s - H x - xi q|| / ||s|| <= tol; >= 0 */
    int64_t max_iters;   /* > 0: row updates (greedy) or iterations (aggregated) */
    uint64_t seed;       /* Philox key word 0 */
    int32_t schedule;    /* vrk_schedule */
    int32_t tile_waves;  /* MFMA engine: waves per workgroup, 0 (auto = 16), 8 or 16.
                            VECTOR engine: 1 selects the small-channel form (one wave per
                            64-antenna slot, at most four, per right-hand side; the
                            channel zero-padded in LDS, x and the per-user state in
                            registers; needs nt <= 1024, k <= 64, interval VRs and the
                            padded channel, 16 ceil(k / 16) rows of 64, 128, 256, 512 or
                            1024 antennas, within 128 KiB), 4 the general form (four waves, any size
                            within LDS), 0, 8 or 16 the small-channel form where it fits.
                            1 or 4 with the AUTO engine selects the VECTOR engine. */
    int32_t persistent;  /* MFMA engine: 1 = one workgroup per resident slot, draining
                            per-XCD work queues (drops assigned by cost); 0 = one
                            workgroup per 16-RHS tile */
    int32_t wave_tiles;  /* MFMA engine, AHK and VR-OAHK: how the waves of a tile share it.
                            -1: block tiles (tile_waves waves split every Gram product of
                            one tile); 1, 2, 4 or 8: wave-owned tiles, that many waves per
                            tile, each owning whole 16-user row blocks (at most 4 each, 2
                            with 8 waves) with its state in registers, several tiles per
                            compute unit, XCD-contiguous work order; 0: auto (wave-owned
                            tiles with two row blocks per wave when tiles x waves per
                            tile >= 4096, every drop has at most 16 chunks of F users
                            and tile_waves, persistent are unset) */
    int32_t check_every; /* the stop rule is tested when the iteration count is a multiple of
                            it (and at max_iters); 0 or 1: every iteration. Later tests only
                            add iterations: the sweeps never increase the error (Lemma 2,
                            Lemma 3), so x stays within the tolerance; iteration counts are
                            multiples of it unless the cap stopped the column. */
} vrk_options;

typedef struct vrk_plan vrk_plan;

/* Fills o with: VR_OAHK, BAIWU, C64, AUTO engine, tol 1e-5,
 * max_iters 100000, seed 0, schedules and tiles auto, check_every 1. */
void vrk_default_options(vrk_options *o);

/* Host only (no device access): validates nprob problems, builds the VR
 * plan of each (overlap sets X_k, the orthogonal set F as a maximum
 * independent set of the interval overlap graph, exact by earliest-end
 * greedy, or of the subarray graph by reducing-peeling; colour classes, tile
 * maps) and reports the workspace size in bytes. *out receives a plan the
 * caller frees with vrk_plan_destroy. The vr_start / vr_len / vr_mask
 * arrays are copied; device pointers are recorded, not read. */
vrk_status vrk_plan_create(const vrk_problem *probs, int32_t nprob, const vrk_options *opt,
                           size_t *ws_bytes, vrk_plan **out);

/* Attaches the caller's device workspace (>= ws_bytes, 256-byte aligned),
 * copies the plan tables into it and enqueues the row-norm and tile-pack
 * kernels on `stream` (a hipStream_t; null = default stream). Reads H.
 * Must be called again if H changes. */
vrk_status vrk_plan_bind(vrk_plan *pl, void *d_ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): vrk_plan_bind with the
 * library's own workspace instead of the caller's. That workspace is one
 * VRK_SCRATCH_BYTES array per device, held from the library's first use of
 * the device until the process ends. The call binds the plan to the array
 * of the current device (make the device the plan's buffers live on current
 * first) and does what vrk_plan_bind does: tables copied in, row-norm and
 * tile kernels enqueued on `stream`; it allocates nothing. Plans whose
 * ws_bytes (from vrk_plan_create) exceed VRK_SCRATCH_BYTES get
 * VRK_EWORKSPACE before anything is enqueued. Every plan bound this way on
 * one device shares the array, and only the latest binding owns it: vrk_solve,
 * vrk_solve_adjoint and vrk_link_metrics of a plan bound earlier return
 * VRK_ESTATE until it is bound again. Work of different plans on that array
 * must not overlap in time: a binding enqueued while another plan's solve on
 * the array may still run (on another stream, or from another thread) races
 * with it. Nothing in the array needs to start zeroed (every kernel writes
 * what it later reads). */
#define VRK_SCRATCH_BYTES ((size_t)64 << 20)
vrk_status vrk_plan_bind_static(vrk_plan *pl, void *stream);

/* After the caller changed the values of H in place (same buffers, same VRs,
 * e.g. a training step on the channel), recomputes on `stream` what a binding
 * derives from H: the row norms ||a_i||^2 = ||H[i, VR_i]||^2 + xi and
 * ||A||_F^2 (Alg. 1 initialisation) and, on the MFMA engine, the packed
 * channel tiles and the Gram tiles of H H^H + xi I. Only enqueues kernels
 * (no copy, no allocation, no synchronisation), so it can be captured into a
 * HIP graph with the solves. VRK_ESTATE before a binding. */
vrk_status vrk_plan_refresh(vrk_plan *pl, void *stream);

/* Enqueues the solve of every right-hand side of every problem. Writes X,
 * V and, when non-null, per-RHS statistics laid out problem after problem
 * (sum of nrhs entries): d_iters (updates done), d_relres (final relative
 * residual), d_flags (bit 0 converged, 1 non-finite, 2 max_iters). */
vrk_status vrk_solve(vrk_plan *pl, void *stream, int32_t *d_iters, float *d_relres,
                     int32_t *d_flags);

/* Implicit-differentiation backward pass of x = H^H (H H^H + xi I)^-1 s,
 * given GX = 2 dL/d conj(x) of a real loss and the X, V of a previous
 * vrk_solve on the same plan: forms b = H g, runs the same Kaczmarz solve
 * on the same system with right-hand side b (mu = its q), then writes
 * GS = mu, *gxi = -Re sum_b mu_b^H v_b and, on VR entries,
 * GH = sum_b v_b (g_b - H^H mu_b)^H - mu_b x_b^H. Statistics as vrk_solve. */
vrk_status vrk_solve_adjoint(vrk_plan *pl, void *stream, int32_t *d_iters, float *d_relres,
                             int32_t *d_flags);

/* Link metrics of RZF precoding (signal model, spectral efficiency and the
 * RZF precoder of the paper, with Remark 1: running the solve on S = I_K
 * gives the precoding matrix column by column). Every problem must have
 * nrhs == k and S = I_K (column b of S the canonical vector e_b), and a
 * vrk_solve on the plan must precede the call: row b of X is then f_b, the
 * unnormalised precoder of user b, F = H^H (H H^H + xi I)^-1. For problem p
 * the call writes (device pointers of out[p], caller-owned):
 *   E[u * lde + b] = h_u^H f_b = sum over n in VR_u of H[u][n] X[b][n]
 *                    (k x k, the plan's complex type, lde >= k),
 *   beta[0]        = 1 / ||F||_F (so that ||beta F||_F = 1, the power budget),
 *   rate[u]        = log2(1 + beta^2 |E_uu|^2 / (beta^2 sum_{b != u} |E_ub|^2 + noise))
 *                    (double, bit/s/Hz), the spectral efficiency of user u under the
 *                    signal model with noise = sigma^2 / rho given per problem (the
 *                    regulariser xi of the plan is not used here: it equals sigma^2 / rho
 *                    only when chosen so; with xi = K sigma^2 / rho, noise = xi / K).
 * On MFMA-engine plans E is evaluated as (H H^H) V^T = (M - xi I) V^T from
 * the plan's Gram tiles and the solve's V (the MFMA solve forms x = H^H v, so
 * this is the same quantity; V is kept in the workspace when the caller
 * passed none); beta is summed from X itself.
 * Asynchronous on stream. The nprob-entry output table is copied to the
 * workspace when it differs from the previous call's on this binding (the
 * workspace belongs to the plan while bound), so repeated calls with the
 * same outputs copy nothing. VRK_EINVAL for a problem with nrhs != k, a
 * null output or a noise that is not finite and > 0; VRK_ESTATE before bind. */
typedef struct {
    void *E;       /* device out, k x k row-major */
    int64_t lde;
    double *rate;  /* device out, k */
    double *beta;  /* device out, 1 */
    double noise;  /* host value: sigma^2 / rho of the rate formula, finite and > 0 */
} vrk_link_out;
vrk_status vrk_link_metrics(vrk_plan *pl, const vrk_link_out *out, void *stream);

/* Autotuner. Picks the execution configuration of a batch by timing it
 * on the device: for complex64 the MFMA engine with 8 or 16 waves per
 * workgroup, each with one workgroup per 16-RHS tile or the persistent
 * per-XCD work queues, and the vector engine with the gather and
 * colour-class schedules; for complex128 the vector engine's two
 * schedules. Each candidate is planned, bound to d_ws, run once and timed
 * over `reps` solves with HIP events on `stream` (the call synchronises
 * the stream; it is not graph-capturable). The caller's X and V are
 * overwritten. On return opt's engine, tile_waves, persistent and schedule
 * hold the fastest candidate and *best_ms its time per
 * solve.
 * With d_ws null nothing runs: *ws_needed gets the workspace size the
 * largest candidate needs. cache_path (nullable) names a text file of
 * previous results keyed by the batch's shape signature (variant, dtype,
 * and per problem Nt, K, B and band size); a hit returns the cached choice
 * without timing, a miss appends the new result. */
vrk_status vrk_autotune(const vrk_problem *probs, int32_t nprob, vrk_options *opt, void *d_ws,
                        size_t ws_bytes, void *stream, const char *cache_path, int32_t reps,
                        size_t *ws_needed, float *best_ms);

/* Plan inspection (host only), for tests and tooling. Writes up to `cap`
 * int32 values of the requested table of problem `prob` into out and
 * returns the table length, or -1 on a bad argument. */
typedef enum {
    VRK_Q_PERM = 0,      /* users sorted by (VR start, end, index) */
    VRK_Q_FSET = 1,      /* orthogonal set F, ascending user index */
    VRK_Q_COLOUR = 2,    /* colour class of each user */
    VRK_Q_XOFF = 3,      /* CSR offsets of X_k, length k + 1 */
    VRK_Q_XIDX = 4,      /* CSR indices of X_k (ascending, includes k) */
    VRK_Q_ENGINE = 5,    /* [engine, schedule, tile_waves, lds_bytes, persistent, grid,
                            (row, column) entries per thread of the MFMA solve,
                            RHS splits of the MFMA adjoint gradient tiles, RHS splits of
                            the blocks of C = sum_b v_b mu_b^H of the MFMA adjoint,
                            tile_waves of the MFMA adjoint solve (8 when every drop has
                            at most 64 users and tile_waves is auto, else tile_waves),
                            waves per wave-owned tile (0: block tiles), row blocks per
                            wave of the wave-owned tiles] */
    VRK_Q_TILES = 6,     /* [residual tiles, aggregation tiles, band entries, Gram tiles] per problem */
    VRK_Q_GRAD = 7       /* MFMA adjoint gradient of the whole plan: [band tiles, RHS splits of a band
                            tile, blocks of C, RHS splits of a C block, runs of the reduction kernel,
                            longest run (band tiles one reduction workgroup takes)]; zeros
                            without adjoint buffers or on the vector engine */
} vrk_query;
int64_t vrk_plan_query(const vrk_plan *pl, int32_t prob, int32_t what, int32_t *out, int64_t cap);

void vrk_plan_destroy(vrk_plan *pl);

const char *vrk_status_string(vrk_status s);
const char *vrk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VRK_H */
