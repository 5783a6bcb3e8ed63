/*
 * FP64 reference ("oracle") for VR-banded Kaczmarz RZF precoding.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may link, load
 * or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code with the HIP path.
 *
 * Plain, slow and written to be checked against the paper by eye:
 * std C11 `double complex`, no blocking, no fusion, no reordering beyond
 * what the cited definitions state. OpenMP appears only as an outer loop
 * over independent right-hand sides, or over users where the gradient sums
 * over right-hand sides (each sum still taken in right-hand-side order).
 *
 * Orientation. H is K x Nt, row-major, row k = what user k sees (the
 * paper's channel matrix is its conjugate transpose). The augmented system
 * (paper Sec. III-B, the consistent system G^H w = s with G = [H; sqrt(xi) I])
 * is A z = s with A = [H, sqrt(xi) I_K], z = [x; u], u = sqrt(xi) q, so row i
 * is a_i^H = [H[i,:], sqrt(xi) e_i^T], ||a_i||^2 = ||H[i,:]||^2 + xi, and the
 * residual is r = s - H x - xi q (Alg. 1, residual step).
 *
 * Visibility region (VR) of user k: the half-open antenna interval
 * [vr_start[k], vr_start[k] + vr_len[k]). Only those entries of H are read.
 * Two users overlap iff max(starts) < min(ends); touching or empty
 * intervals are disjoint (Lemma 1: disjoint VRs give orthogonal rows).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Status / flag values (mirrored in oracle/__init__.py). */
enum { ORC_OK = 0, ORC_EINVAL = 1 };
enum { ORC_GRK = 0, ORC_AHK = 1, ORC_VR_OGRK = 2, ORC_VR_OAHK = 3 };
enum { ORC_SEL_BAIWU = 0, ORC_SEL_RESIDUAL = 1, ORC_SEL_MAX = 2, ORC_SEL_ENERGY = 3, ORC_SEL_UNIFORM = 4 };
enum { ORC_F_CONVERGED = 1, ORC_F_NONFINITE = 2, ORC_F_MAXITER = 4 };

/* One channel drop. */
typedef struct {
    int32_t nt, k;
    double xi;
    const cplx *H;          /* K x Nt, row stride ldh */
    int64_t ldh;
    const int32_t *vs, *vl; /* VR start / length per user */
    const uint64_t *mask;   /* null, or per user the visible subarrays (bit s) */
    int32_t n_sub;          /* subarrays S of Nt / S antennas each (with mask) */
} orc_problem;

static inline int32_t vr_end(const orc_problem *p, int i) { return p->vs[i] + p->vl[i]; }

/* Antenna n is in user k's VR: inside [vs, ve) and, with subarray masks,
 * on a subarray of M_k (the indicator u_k of the subarray VR model, Sec. II).
 * Loops below run over [vs, ve) and skip the antennas this rejects. */
static inline int seen(const orc_problem *p, int k, int32_t n)
{
    return !p->mask || ((p->mask[k] >> (n / (p->nt / p->n_sub))) & 1u);
}

static int validate(const orc_problem *p)
{
    if (!p || p->nt < 1 || p->k < 1 || !(p->xi > 0.0) || !isfinite(p->xi) || !p->H ||
        p->ldh < p->nt || !p->vs || !p->vl)
        return ORC_EINVAL;
    for (int i = 0; i < p->k; ++i)
        if (p->vs[i] < 0 || p->vl[i] < 0 || (int64_t)p->vs[i] + p->vl[i] > p->nt)
            return ORC_EINVAL;
    if (p->mask) {
        /* [vs, ve) must be the hull of the visible subarrays */
        if (p->n_sub < 1 || p->n_sub > 64 || p->nt % p->n_sub) return ORC_EINVAL;
        const int32_t L = p->nt / p->n_sub;
        for (int i = 0; i < p->k; ++i) {
            uint64_t m = p->mask[i];
            if (p->n_sub < 64 && (m >> p->n_sub)) return ORC_EINVAL;
            int32_t lo = 0, hi = 0;
            if (m) {
                int s0 = 0, s1 = p->n_sub - 1;
                while (!((m >> s0) & 1u)) ++s0;
                while (!((m >> s1) & 1u)) --s1;
                lo = s0 * L;
                hi = (s1 + 1) * L;
            }
            if (p->vs[i] != lo || vr_end(p, i) != hi) return ORC_EINVAL;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11). Ten rounds of the
 * 4x64 S-box with the published multipliers and Weyl key increments.
 * The selection step draws u = (out[0] >> 40) * 2^-24 with key (seed, 0)
 * and counter (step, rhs, drop, 0); the paper leaves the RNG unspecified.
 * ---------------------------------------------------------------------- */
static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_uniform24(uint64_t seed, int64_t step, int64_t rhs, int64_t drop)
{
    uint64_t ctr[4] = {(uint64_t)step, (uint64_t)rhs, (uint64_t)drop, 0};
    uint64_t key[2] = {seed, 0}, out[4];
    orc_philox4x64_10(ctr, key, out);
    return (double)(out[0] >> 40) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------
 * VR structure (Sec. IV-B and V-B).
 * ---------------------------------------------------------------------- */
static int vr_overlap(const orc_problem *p, int i, int j)
{
    if (p->mask) return (p->mask[i] & p->mask[j]) != 0;   /* |M_i cap M_j| > 0 */
    int32_t lo = p->vs[i] > p->vs[j] ? p->vs[i] : p->vs[j];
    int32_t hi = vr_end(p, i) < vr_end(p, j) ? vr_end(p, i) : vr_end(p, j);
    return lo < hi;
}

/* Non-orthogonal set X_k of Sec. IV-B: users whose VR overlaps user k's,
 * including k itself. CSR: xoff[K+1], xidx[<= K*K], indices ascending. */
int orc_overlap_sets(const orc_problem *p, int32_t *xoff, int32_t *xidx)
{
    if (validate(p)) return ORC_EINVAL;
    int32_t n = 0;
    for (int k = 0; k < p->k; ++k) {
        xoff[k] = n;
        for (int j = 0; j < p->k; ++j)
            if (j == k || vr_overlap(p, k, j)) xidx[n++] = j;
    }
    xoff[p->k] = n;
    return ORC_OK;
}

/* Orthogonal set F: a maximum independent set of the VR overlap graph
 * (problem max_set of Sec. V-B). With subarray masks see
 * mis_reducing_peeling below. For contiguous VRs the graph is an
 * interval graph, on which the earliest-end greedy is exact: visit users by
 * (end, start, index) and keep one whose start is at or after the end of
 * the last kept one. Users with an empty VR overlap nobody and are always
 * kept. Output: in_f[k] = 1 for k in F. */
/* (end, start, index) order used by the greedy. */
static int before_by_end(const orc_problem *p, int i, int j)
{
    if (vr_end(p, i) != vr_end(p, j)) return vr_end(p, i) < vr_end(p, j);
    if (p->vs[i] != p->vs[j]) return p->vs[i] < p->vs[j];
    return i < j;
}

/* F on the general VR graph of the subarray model (edge iff the masks
 * share a subarray), where maximum independent set is hard: the
 * reducing-peeling heuristic of the linear-time method the paper cites for
 * problem max_set. While vertices remain: a vertex of degree 0 joins F; else
 * a vertex of degree 1 joins F and its neighbour is deleted (both exact
 * reductions); else a vertex of largest degree is peeled (deleted). Degrees
 * count remaining vertices; ties go to the smallest index. Afterwards the
 * peeled vertices, latest first, join F when no neighbour is in it, so F is
 * maximal. */
static void mis_reducing_peeling(const orc_problem *p, uint8_t *in_f)
{
    const int K = p->k;
    uint8_t *alive = malloc(K);
    int *peeled = malloc(sizeof(int) * K), np = 0;
    for (int v = 0; v < K; ++v) { alive[v] = 1; in_f[v] = 0; }
    for (;;) {
        int pick0 = -1, pick1 = -1, pickp = -1, dmax = -1;
        for (int v = 0; v < K; ++v) {
            if (!alive[v]) continue;
            int d = 0;
            for (int u = 0; u < K; ++u)
                if (u != v && alive[u] && vr_overlap(p, u, v)) ++d;
            if (d == 0 && pick0 < 0) pick0 = v;
            if (d == 1 && pick1 < 0) pick1 = v;
            if (d > dmax) { dmax = d; pickp = v; }
        }
        if (pickp < 0) break;                  /* nothing left */
        if (pick0 >= 0) { in_f[pick0] = 1; alive[pick0] = 0; continue; }
        if (pick1 >= 0) {
            in_f[pick1] = 1;
            alive[pick1] = 0;
            for (int u = 0; u < K; ++u)
                if (u != pick1 && alive[u] && vr_overlap(p, u, pick1)) alive[u] = 0;
            continue;
        }
        alive[pickp] = 0;
        peeled[np++] = pickp;
    }
    for (int t = np - 1; t >= 0; --t) {
        int v = peeled[t], free_v = 1;
        for (int u = 0; u < K && free_v; ++u)
            if (in_f[u] && vr_overlap(p, u, v)) free_v = 0;
        if (free_v) in_f[v] = 1;
    }
    free(alive);
    free(peeled);
}

int orc_mis(const orc_problem *p, uint8_t *in_f)
{
    if (validate(p)) return ORC_EINVAL;
    if (p->mask) { mis_reducing_peeling(p, in_f); return ORC_OK; }
    int *ord = malloc(sizeof(int) * p->k);
    int n = 0;
    for (int k = 0; k < p->k; ++k) {
        in_f[k] = 0;
        if (p->vl[k] == 0) in_f[k] = 1; else ord[n++] = k;
    }
    for (int a = 1; a < n; ++a) {          /* insertion sort by (end, start, index) */
        int key = ord[a], b = a - 1;
        while (b >= 0 && before_by_end(p, key, ord[b])) { ord[b + 1] = ord[b]; --b; }
        ord[b + 1] = key;
    }
    int32_t last_end = INT32_MIN;
    for (int t = 0; t < n; ++t) {
        int k = ord[t];
        if (p->vs[k] >= last_end) { in_f[k] = 1; last_end = vr_end(p, k); }
    }
    free(ord);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Closed-form RZF (precoding equation of Sec. II-C; Theorem 1, Remark 1):
 *   v = (H H^H + xi I)^-1 s,   x = H^H v.
 * Gram matrix over overlapping VRs, textbook Cholesky M = L L^H
 * (Golub & Van Loan), forward and back substitution, then x = H^H v.
 * ---------------------------------------------------------------------- */
static void gram(const orc_problem *p, cplx *M)
{
    const int K = p->k;
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
            cplx acc = 0;
            int32_t lo = p->vs[i] > p->vs[j] ? p->vs[i] : p->vs[j];
            int32_t hi = vr_end(p, i) < vr_end(p, j) ? vr_end(p, i) : vr_end(p, j);
            for (int32_t n = lo; n < hi; ++n)
                if (seen(p, i, n) && seen(p, j, n))
                    acc += p->H[i * p->ldh + n] * conj(p->H[j * p->ldh + n]);
            M[i * K + j] = acc + (i == j ? p->xi : 0.0);
        }
}

static int cholesky(int K, const cplx *M, cplx *L)
{
    memset(L, 0, sizeof(cplx) * K * K);
    for (int j = 0; j < K; ++j) {
        double d = creal(M[j * K + j]);
        for (int t = 0; t < j; ++t) d -= creal(L[j * K + t] * conj(L[j * K + t]));
        if (!(d > 0.0)) return ORC_EINVAL;
        double ljj = sqrt(d);
        L[j * K + j] = ljj;
        for (int i = j + 1; i < K; ++i) {
            cplx acc = M[i * K + j];
            for (int t = 0; t < j; ++t) acc -= L[i * K + t] * conj(L[j * K + t]);
            L[i * K + j] = acc / ljj;
        }
    }
    return ORC_OK;
}

static void chol_solve(int K, const cplx *L, const cplx *b, cplx *v)
{
    cplx *y = malloc(sizeof(cplx) * K);
    for (int i = 0; i < K; ++i) {            /* L y = b */
        cplx acc = b[i];
        for (int t = 0; t < i; ++t) acc -= L[i * K + t] * y[t];
        y[i] = acc / L[i * K + i];
    }
    for (int i = K - 1; i >= 0; --i) {       /* L^H v = y */
        cplx acc = y[i];
        for (int t = i + 1; t < K; ++t) acc -= conj(L[t * K + i]) * v[t];
        v[i] = acc / L[i * K + i];
    }
    free(y);
}

/* x = H^H v over the VR bands. */
static void apply_hh(const orc_problem *p, const cplx *v, cplx *x)
{
    for (int n = 0; n < p->nt; ++n) x[n] = 0;
    for (int k = 0; k < p->k; ++k)
        for (int32_t n = p->vs[k]; n < vr_end(p, k); ++n)
            if (seen(p, k, n))
                x[n] += conj(p->H[k * p->ldh + n]) * v[k];
}

/* b = H g over the VR bands. */
static void apply_h(const orc_problem *p, const cplx *g, cplx *b)
{
    for (int k = 0; k < p->k; ++k) {
        cplx acc = 0;
        for (int32_t n = p->vs[k]; n < vr_end(p, k); ++n)
            if (seen(p, k, n)) acc += p->H[k * p->ldh + n] * g[n];
        b[k] = acc;
    }
}

/* S: B x K (row stride lds); X: B x Nt (ldx); V: B x K (ldv), V nullable. */
int orc_rzf_cholesky(const orc_problem *p, int32_t nrhs, const cplx *S, int64_t lds,
                     cplx *X, int64_t ldx, cplx *V, int64_t ldv)
{
    if (validate(p) || nrhs < 0 || lds < p->k || ldx < p->nt || (V && ldv < p->k)) return ORC_EINVAL;
    const int K = p->k;
    cplx *M = malloc(sizeof(cplx) * K * K), *L = malloc(sizeof(cplx) * K * K);
    gram(p, M);
    int st = cholesky(K, M, L);
    if (st == ORC_OK) {
#pragma omp parallel for schedule(static)
        for (int b = 0; b < nrhs; ++b) {
            cplx *v = malloc(sizeof(cplx) * K);
            chol_solve(K, L, S + (int64_t)b * lds, v);
            apply_hh(p, v, X + (int64_t)b * ldx);
            if (V) memcpy(V + (int64_t)b * ldv, v, sizeof(cplx) * K);
            free(v);
        }
    }
    free(M); free(L);
    return st;
}

/* Closed-form gradient of a real loss through x = H^H (H H^H + xi I)^-1 s,
 * given G = the incoming gradient on X in the 2 dL/d(conj x) convention:
 *   mu = M^-1 H g,  xh = H^H mu,
 *   dL/ds = mu,  dL/dxi = -Re sum_b mu_b^H v_b,
 *   dL/dH = sum_b v_b (g_b - xh_b)^H - mu_b x_b^H   (VR band entries only;
 * the entries outside the band are fixed zeros of the channel equation).
 * gH: K x Nt (ldgh), entries outside the bands are written as 0. */
int orc_rzf_grad(const orc_problem *p, int32_t nrhs, const cplx *S, int64_t lds,
                 const cplx *G, int64_t ldg, cplx *gH, int64_t ldgh, cplx *gS, int64_t ldgs,
                 double *gxi)
{
    if (validate(p) || nrhs < 0 || lds < p->k || ldg < p->nt || ldgh < p->nt || ldgs < p->k)
        return ORC_EINVAL;
    const int K = p->k, N = p->nt;
    cplx *M = malloc(sizeof(cplx) * K * K), *L = malloc(sizeof(cplx) * K * K);
    gram(p, M);
    int st = cholesky(K, M, L);
    if (st != ORC_OK) { free(M); free(L); return st; }
    /* per right-hand side (independent): v_b, x_b, mu_b, xh_b */
    cplx *Vb = malloc(sizeof(cplx) * (size_t)nrhs * K), *Xb = malloc(sizeof(cplx) * (size_t)nrhs * N);
    cplx *MUb = malloc(sizeof(cplx) * (size_t)nrhs * K), *XHb = malloc(sizeof(cplx) * (size_t)nrhs * N);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < nrhs; ++b) {
        const cplx *s = S + (int64_t)b * lds, *g = G + (int64_t)b * ldg;
        cplx *v = Vb + (size_t)b * K, *x = Xb + (size_t)b * N;
        cplx *mu = MUb + (size_t)b * K, *xh = XHb + (size_t)b * N;
        cplx *hg = malloc(sizeof(cplx) * K);
        chol_solve(K, L, s, v);
        apply_hh(p, v, x);
        apply_h(p, g, hg);
        chol_solve(K, L, hg, mu);
        apply_hh(p, mu, xh);
        free(hg);
    }
    /* sums over the right-hand sides, b = 0, 1, ... in order for every entry
     * (users are independent, so they may run in parallel) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < K; ++k) {
        for (int n = 0; n < N; ++n) gH[k * ldgh + n] = 0;
        for (int b = 0; b < nrhs; ++b) {
            const cplx *g = G + (int64_t)b * ldg, *x = Xb + (size_t)b * N, *xh = XHb + (size_t)b * N;
            const cplx vk = Vb[(size_t)b * K + k], muk = MUb[(size_t)b * K + k];
            for (int32_t n = p->vs[k]; n < vr_end(p, k); ++n)
                if (seen(p, k, n))
                    gH[k * ldgh + n] += vk * conj(g[n] - xh[n]) - muk * conj(x[n]);
        }
    }
    double acc_xi = 0.0;
    for (int b = 0; b < nrhs; ++b)
        for (int k = 0; k < K; ++k) {
            const cplx mu = MUb[(size_t)b * K + k];
            gS[(int64_t)b * ldgs + k] = mu;
            acc_xi -= creal(conj(mu) * Vb[(size_t)b * K + k]);
        }
    *gxi = acc_xi;
    free(Vb); free(Xb); free(MUb); free(XHb); free(M); free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Kaczmarz primitives on A z = s, z = [x; u], u = sqrt(xi) q. The state is
 * kept as (x, q) exactly as in Alg. 1 (m and q there).
 * ---------------------------------------------------------------------- */

/* ||a_i||^2 = ||H[i, VR_i]||^2 + xi   (Alg. 1, stored row norms). */
static double row_norm2(const orc_problem *p, int i)
{
    double acc = 0.0;
    for (int32_t n = p->vs[i]; n < vr_end(p, i); ++n) {
        if (!seen(p, i, n)) continue;
        cplx h = p->H[i * p->ldh + n];
        acc += creal(h) * creal(h) + cimag(h) * cimag(h);
    }
    return acc + p->xi;
}

/* r_i = s_i - a_i^H z = s_i - H[i, VR_i] x[VR_i] - xi q_i   (Alg. 1 residual
 * step; the VR-restricted inner product of Sec. IV-B). */
static cplx residual_row(const orc_problem *p, int i, const cplx *s, const cplx *x, const cplx *q)
{
    cplx acc = 0;
    for (int32_t n = p->vs[i]; n < vr_end(p, i); ++n)
        if (seen(p, i, n)) acc += p->H[i * p->ldh + n] * x[n];
    return s[i] - acc - p->xi * q[i];
}

/* Single-row projection, equation (update):
 *   gamma = r_i / ||a_i||^2,  x += gamma conj(H[i,:]),  q_i += gamma. */
static void project_row(const orc_problem *p, int i, cplx r_i, double nrm_i, cplx *x, cplx *q)
{
    cplx gamma = r_i / nrm_i;
    for (int32_t n = p->vs[i]; n < vr_end(p, i); ++n)
        if (seen(p, i, n)) x[n] += gamma * conj(p->H[i * p->ldh + n]);
    q[i] += gamma;
}

/* Aggregated-hyperplane projection, equation (update4) with the aggregation
 * coefficients (coefficient) restricted to the user set `in_set`:
 *   phi_i = r_i / ||a_i||^2 (i in set, else 0),
 *   A^H phi = [H^H phi; sqrt(xi) phi],
 *   gamma = phi^H r / ||A^H phi||^2 = (sum |r_i|^2/||a_i||^2) / (||H^H phi||^2 + xi ||phi||^2),
 *   x += gamma H^H phi,  q += gamma phi.
 * r holds the residuals of the set's rows at the current iterate. Returns 0
 * when the set's residual is zero (no move). */
static int project_aggregate(const orc_problem *p, const uint8_t *in_set, const cplx *r,
                             const double *nrm, cplx *x, cplx *q, cplx *phi, cplx *hphi)
{
    double num = 0.0, phin = 0.0;
    for (int i = 0; i < p->k; ++i) {
        phi[i] = in_set[i] ? r[i] / nrm[i] : 0.0;
        num += creal(conj(phi[i]) * r[i]);
        phin += creal(phi[i] * conj(phi[i]));
    }
    if (!(num > 0.0)) return 0;
    apply_hh(p, phi, hphi);
    double den = 0.0;
    for (int n = 0; n < p->nt; ++n) den += creal(hphi[n] * conj(hphi[n]));
    den += p->xi * phin;
    double gamma = num / den;
    for (int n = 0; n < p->nt; ++n) x[n] += gamma * hphi[n];
    for (int i = 0; i < p->k; ++i) q[i] += gamma * phi[i];
    return 1;
}

/* Orthogonal-set projection, Proposition 1 (orthogonal): for pairwise
 * disjoint VRs the aggregated step has gamma = 1, so each row of the set
 * adds phi_i a_i independently. */
static void project_orthogonal(const orc_problem *p, const uint8_t *in_f, const cplx *r,
                               const double *nrm, cplx *x, cplx *q)
{
    for (int i = 0; i < p->k; ++i)
        if (in_f[i]) {
            cplx phi = r[i] / nrm[i];
            for (int32_t n = p->vs[i]; n < vr_end(p, i); ++n)
                if (seen(p, i, n)) x[n] += phi * conj(p->H[i * p->ldh + n]);
            q[i] += phi;
        }
}

/* Row selection of the single-row sweeps (GRK / VR-OGRK, Sec. IV-A; the
 * randomized Kaczmarz criteria of Sec. III-A). Returns the chosen row.
 *  RESIDUAL: p_i = |r_i|^2 / ||r||^2 (the printed GRK rule).
 *  BAIWU: the greedy randomized rule the paper cites (Bai & Wu 2018):
 *    eps = (max_i |r_i|^2/||a_i||^2 / ||r||^2 + 1/||A||_F^2) / 2,
 *    U = {i : |r_i|^2 >= eps ||r||^2 ||a_i||^2}, p_i ~ |r_i|^2 on U.
 *    Written as rho_i = |r_i|^2/||a_i||^2 >= theta with
 *    theta = min(rho_max, (rho_max + ||r||^2/||A||_F^2)/2).
 *  MAX: argmax_i |r_i|^2/||a_i||^2, lowest index on ties (the greedy
 *    Kaczmarz benchmark).
 *  ENERGY: p_i = ||a_i||^2 / ||A||_F^2, the energy criterion of the
 *    randomized Kaczmarz method (Sec. III-A); the residual plays no part.
 *  UNIFORM: p_i = 1/K, the uniform criterion (Sec. III-A; URK of Table I).
 * Sampling: smallest i whose inclusive prefix of weights (index order)
 * exceeds u * W, W = the prefix total; if rounding leaves none, the last
 * index of positive weight. */
static int select_row(int K, int rule, const cplx *r, const double *nrm, double fro2, double u)
{
    if (rule == ORC_SEL_ENERGY || rule == ORC_SEL_UNIFORM) {
        double W = 0.0;
        for (int i = 0; i < K; ++i) W += rule == ORC_SEL_ENERGY ? nrm[i] : 1.0;
        double target = u * W, acc = 0.0;
        for (int i = 0; i < K; ++i) {
            acc += rule == ORC_SEL_ENERGY ? nrm[i] : 1.0;
            if (acc > target) return i;
        }
        return K - 1;
    }
    double rr = 0.0, rho_max = -1.0;
    int imax = 0;
    for (int i = 0; i < K; ++i) {
        double w = creal(r[i]) * creal(r[i]) + cimag(r[i]) * cimag(r[i]);
        double rho = w / nrm[i];
        rr += w;
        if (rho > rho_max) { rho_max = rho; imax = i; }
    }
    if (rule == ORC_SEL_MAX) return imax;
    double theta = 0.0;
    if (rule == ORC_SEL_BAIWU) {
        theta = 0.5 * (rho_max + rr / fro2);
        if (theta > rho_max) theta = rho_max;
    }
    double *pre = malloc(sizeof(double) * K);
    double acc = 0.0;
    int last_pos = imax;
    for (int i = 0; i < K; ++i) {
        double w = creal(r[i]) * creal(r[i]) + cimag(r[i]) * cimag(r[i]);
        int in_u = (rule == ORC_SEL_RESIDUAL) || (w / nrm[i] >= theta);
        if (in_u && w > 0.0) { acc += w; last_pos = i; }
        pre[i] = acc;
    }
    double target = u * acc;
    int pick = last_pos;
    for (int i = 0; i < K; ++i)
        if (pre[i] > target) { pick = i; break; }
    free(pre);
    return pick;
}

static double norm2v(int n, const cplx *v)
{
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return a;
}

/* One right-hand side, one variant, from z = 0 (Alg. 1 initialisation).
 *   GRK     (Sec. IV-A): every step recomputes all residuals from x, checks
 *           the stop rule, selects a row, projects onto it.
 *   VR-OGRK (Alg. 2): starts from r = s; after projecting row i only the
 *           rows of X_i are recomputed from x (Theorem 2 leaves the others
 *           unchanged); selection as GRK on the maintained residual.
 *   AHK     (Sec. V-A): every iteration the full residual, then one
 *           aggregated projection over all rows.
 *   VR-OAHK (Alg. 3): every iteration the full residual (stop check), the
 *           orthogonal half-step on F with gamma = 1 (Prop. 1), the residual
 *           of V from the half-updated x, and an aggregated projection over V.
 * Stop rule: ||r||_2 / ||s||_2 <= tol, tested before every update on the
 * residual the variant holds. iters = updates done (rows for GRK/VR-OGRK,
 * iterations for AHK/VR-OAHK). flags: 1 converged, 2 non-finite, 4 hit
 * max_iters. s = 0 gives x = 0 after 0 updates.
 * Trace (optional): z after every update (and every half-step of VR-OAHK),
 * as rows of Nt + K entries [x; q], starting with z0; trace_idx gets the
 * chosen row per step (GRK family) or -1 / -2 for the F / V half-steps. */
int orc_kaczmarz(const orc_problem *p, int variant, int rule, double tol, int64_t max_iters,
                 uint64_t seed, int64_t drop, int64_t rhs, const cplx *s,
                 cplx *x, cplx *q, int64_t *iters, double *relres, int32_t *flags,
                 cplx *trace_z, int32_t *trace_idx, int64_t trace_cap, int64_t *trace_n)
{
    if (validate(p) || variant < 0 || variant > 3 || rule < 0 || rule > 4 || !(tol >= 0.0) ||
        max_iters < 0)
        return ORC_EINVAL;
    const int K = p->k, N = p->nt;
    double *nrm = malloc(sizeof(double) * K);
    cplx *r = malloc(sizeof(cplx) * K), *phi = malloc(sizeof(cplx) * K);
    cplx *hphi = malloc(sizeof(cplx) * N);
    uint8_t *all = malloc(K), *in_f = malloc(K), *in_v = malloc(K);
    int32_t *xoff = malloc(sizeof(int32_t) * (K + 1)), *xidx = malloc(sizeof(int32_t) * K * K);
    double fro2 = 0.0;
    for (int i = 0; i < K; ++i) { nrm[i] = row_norm2(p, i); fro2 += nrm[i]; all[i] = 1; }
    orc_overlap_sets(p, xoff, xidx);
    orc_mis(p, in_f);
    for (int i = 0; i < K; ++i) in_v[i] = !in_f[i];
    for (int n = 0; n < N; ++n) x[n] = 0;
    for (int i = 0; i < K; ++i) { q[i] = 0; r[i] = s[i]; }   /* z0 = 0, r0 = s */

    int64_t tn = 0;
#define TRACE(idx)                                                            \
    do {                                                                      \
        if (trace_z && tn < trace_cap) {                                      \
            memcpy(trace_z + tn * (N + K), x, sizeof(cplx) * N);              \
            memcpy(trace_z + tn * (N + K) + N, q, sizeof(cplx) * K);          \
            if (trace_idx) trace_idx[tn] = (idx);                             \
        }                                                                     \
        ++tn;                                                                 \
    } while (0)
    TRACE(-3);

    double snorm = sqrt(norm2v(K, s));
    int32_t fl = 0;
    int64_t t = 0;
    double rel = 0.0;
    if (!isfinite(snorm) || !isfinite(fro2)) fl |= ORC_F_NONFINITE;
    else if (snorm == 0.0) { fl |= ORC_F_CONVERGED; rel = 0.0; }
    else {
        for (;;) {
            /* residual the variant holds at the current iterate */
            if (variant != ORC_VR_OGRK)
                for (int i = 0; i < K; ++i) r[i] = residual_row(p, i, s, x, q);
            double rn = sqrt(norm2v(K, r));
            rel = rn / snorm;
            if (!isfinite(rel)) { fl |= ORC_F_NONFINITE; break; }
            if (rel <= tol) { fl |= ORC_F_CONVERGED; break; }
            if (t >= max_iters) { fl |= ORC_F_MAXITER; break; }
            if (variant == ORC_GRK || variant == ORC_VR_OGRK) {
                double u = orc_uniform24(seed, t, rhs, drop);
                int i = select_row(K, rule, r, nrm, fro2, u);
                /* gamma from r_i at the current iterate (Alg. 1 residual step);
                 * for VR-OGRK the held r_i equals it exactly, since x changed
                 * only outside VR_i since it was last recomputed. */
                project_row(p, i, r[i], nrm[i], x, q);
                if (variant == ORC_VR_OGRK)
                    for (int32_t c = xoff[i]; c < xoff[i + 1]; ++c) {
                        int j = xidx[c];
                        r[j] = residual_row(p, j, s, x, q);
                    }
                TRACE(i);
            } else if (variant == ORC_AHK) {
                project_aggregate(p, all, r, nrm, x, q, phi, hphi);
                TRACE(-2);
            } else { /* VR-OAHK */
                project_orthogonal(p, in_f, r, nrm, x, q);
                TRACE(-1);
                for (int i = 0; i < K; ++i)
                    if (in_v[i]) r[i] = residual_row(p, i, s, x, q);
                project_aggregate(p, in_v, r, nrm, x, q, phi, hphi);
                TRACE(-2);
            }
            ++t;
        }
    }
#undef TRACE
    *iters = t;
    *relres = rel;
    *flags = fl;
    if (trace_n) *trace_n = tn;
    free(nrm); free(r); free(phi); free(hphi); free(all); free(in_f); free(in_v);
    free(xoff); free(xidx);
    return ORC_OK;
}

/* Many right-hand sides of one drop (independent; OpenMP over b). */
int orc_kaczmarz_batch(const orc_problem *p, int variant, int rule, double tol, int64_t max_iters,
                       uint64_t seed, int64_t drop, int32_t nrhs, const cplx *S, int64_t lds,
                       cplx *X, int64_t ldx, cplx *V, int64_t ldv, int64_t *iters, double *relres,
                       int32_t *flags)
{
    if (validate(p) || nrhs < 0 || lds < p->k || ldx < p->nt || ldv < p->k) return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int b = 0; b < nrhs; ++b) {
        int st = orc_kaczmarz(p, variant, rule, tol, max_iters, seed, drop, b, S + (int64_t)b * lds,
                              X + (int64_t)b * ldx, V + (int64_t)b * ldv, iters + b, relres + b,
                              flags + b, NULL, NULL, 0, NULL);
        bad |= st;
    }
    return bad ? ORC_EINVAL : ORC_OK;
}

/* Primitives exported for the invariant tests (Theorem 2, Theorem 4,
 * Proposition 1, and the phi = e_i reduction of (update4)). */
void orc_residual_rows(const orc_problem *p, const cplx *s, const cplx *x, const cplx *q, cplx *r)
{
    for (int i = 0; i < p->k; ++i) r[i] = residual_row(p, i, s, x, q);
}

void orc_row_norms(const orc_problem *p, double *nrm)
{
    for (int i = 0; i < p->k; ++i) nrm[i] = row_norm2(p, i);
}

void orc_step_row(const orc_problem *p, int i, const cplx *s, cplx *x, cplx *q)
{
    project_row(p, i, residual_row(p, i, s, x, q), row_norm2(p, i), x, q);
}

void orc_step_orthogonal(const orc_problem *p, const uint8_t *in_f, const cplx *s, cplx *x, cplx *q)
{
    double *nrm = malloc(sizeof(double) * p->k);
    cplx *r = malloc(sizeof(cplx) * p->k);
    for (int i = 0; i < p->k; ++i) { nrm[i] = row_norm2(p, i); r[i] = residual_row(p, i, s, x, q); }
    project_orthogonal(p, in_f, r, nrm, x, q);
    free(nrm); free(r);
}

int orc_step_aggregate(const orc_problem *p, const uint8_t *in_set, const cplx *s, cplx *x, cplx *q)
{
    double *nrm = malloc(sizeof(double) * p->k);
    cplx *r = malloc(sizeof(cplx) * p->k), *phi = malloc(sizeof(cplx) * p->k);
    cplx *hphi = malloc(sizeof(cplx) * p->nt);
    for (int i = 0; i < p->k; ++i) { nrm[i] = row_norm2(p, i); r[i] = residual_row(p, i, s, x, q); }
    int moved = project_aggregate(p, in_set, r, nrm, x, q, phi, hphi);
    free(nrm); free(r); free(phi); free(hphi);
    return moved;
}

int orc_select(int K, int rule, const cplx *r, const double *nrm, double fro2, double u)
{
    return select_row(K, rule, r, nrm, fro2, u);
}

/* Threads an OpenMP parallel region of this library uses (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of later parallel regions (timing only). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
