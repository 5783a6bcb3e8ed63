// Host side of libvrk: argument validation, the VR plan of each problem,
// workspace carving, table upload and kernel dispatch.
//
// The VR plan follows the VR-structure passages of the paper:
//  * overlap sets X_k (Sec. IV-B): users whose VR intersects user k's,
//    including k; Lemma 1 makes every other row orthogonal to row k;
//  * the orthogonal set F (Sec. V-B, problem max_set): a maximum independent
//    set of the VR overlap graph. Contiguous VRs make it an interval graph,
//    where the earliest-end greedy is exact; V is the complement;
//  * colour classes: a minimum partition of the users into sets of pairwise
//    disjoint VRs (optimal interval-graph colouring), used as the group
//    schedule of concurrent row updates (Prop. 1 generalised to every class).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <queue>
#include <set>
#include <string>
#include <vector>

#include "../../include/vrk.h"
#include "kernels.h"
#include "vrk_desc.h"

namespace {

thread_local std::string g_err;

vrk_status fail(vrk_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

vrk_status hip_fail(hipError_t e, const char *what)
{
    return fail(VRK_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return o;
    }
};

struct ProbPlan {
    vrk_problem p{};
    std::vector<int32_t> vs, ve, perm, pos, xoff, xidx, flist, vlist, colour, col_off, col_users;
    std::vector<int32_t> gb_off, gb_users;
    std::vector<uint8_t> inf;
    int32_t ncol = 0;
    // MFMA tables
    int32_t nub = 0, nab = 0, ntile = 0;
    std::vector<int32_t> rab_lo, rab_hi, ag_off, ag_uc, gm_off, gm_c, gm_nf, fpos;
    int32_t nmf = 0;   // columns of MF (F users) when the solve takes the F half-step on the VALU
    std::vector<int32_t> cp_off, cp_col, cp_tr, cp_diag;   // blocks of C on the Gram block pattern
    std::vector<uint64_t> mask;   // subarray masks (empty: interval VRs)
    bool keep_v = false;          // V goes to the workspace (caller gave none; adjoint or S = I_K shape)
    bool stage_h = false;         // vector engine: H's VR entries staged in LDS
    std::vector<int32_t> gaps;    // (user, first antenna, length) of hidden runs inside the hulls
    std::vector<int32_t> fch;     // 4-user chunks (VR-start order) holding a user of F, ascending
    std::vector<int32_t> gm_fs;   // per Gram list entry: its chunk's index in fch, else VRK_WAVE_FCHUNKS
    std::vector<int64_t> ha_off;
    int64_t n_ha = 0, n_hg = 0, n_gm = 0, band = 0;
    // workspace offsets
    size_t o_vs, o_ve, o_xoff, o_xidx, o_flist, o_vlist, o_inf, o_coloff, o_colusr, o_gboff,
        o_gbusr, o_perm, o_pos, o_nrm, o_fro2, o_rablo, o_rabhi, o_haoff, o_agoff, o_aguc,
        o_ha, o_hg, o_sadj, o_xadj, o_vfwd, o_vsrt = 0, o_msrt = 0;
    int64_t rhs_base = 0;
    size_t o_gmoff = 0, o_gmc = 0, o_gm = 0, o_gmnf = 0, o_fpos = 0, o_mf = 0;
    size_t o_cpoff = 0, o_cpcol = 0, o_cptr = 0, o_cpdiag = 0, o_cblk = 0, o_gaps = 0, o_mask = 0, o_fch = 0,
           o_gmfs = 0;
};

}  // namespace

struct vrk_plan {
    vrk_options opt{};
    std::vector<ProbPlan> pp;
    int32_t engine = VRK_ENGINE_VECTOR, schedule = VRK_SCHED_GATHER, waves = 8, ep = 0;
    size_t lds = 0;
    // vector engine: one wave per right-hand side (the single-wave form)
    bool small = false;
    int32_t max_nt = 0;
    // MFMA engine: the adjoint solve's tile shape (8 waves when every drop has
    // at most 64 users and the tile size is left to the plan, else the same)
    int32_t waves_adj = 8, ep_adj = 0, grid_adj = 0;
    size_t lds_adj = 0;
    // MFMA engine, wave-owned tiles (AHK, VR-OAHK): waves per tile and row
    // blocks per wave (0: block tiles), LDS per tile
    int32_t wave_T = 0, wave_bpw = 0;
    size_t lds_wave = 0;
    size_t table_end = 0, ws_bytes = 0, o_desc = 0, o_work = 0;
    int64_t total_rhs = 0, max_tiles = 0;
    int32_t max_rhs = 0, max_k = 0;
    bool adjoint_ready = false;
    bool any_gaps = false;      // some problem has hidden antennas inside a hull
    std::vector<VrkWork> work;
    std::vector<int4> gtiles;   // band tiles of the adjoint gradient (MFMA engine)
    size_t o_gtiles = 0;
    int32_t qbase[VRK_NQUEUE] = {0}, qsize[VRK_NQUEUE] = {0};
    size_t o_queue = 0;         // int32 counters[8], base[8], size[8]
    int32_t gsplit = 1;         // RHS splits of the adjoint gradient tiles
    size_t o_gpart = 0;
    std::vector<int4> ctiles;   // (problem, C block, split, row block) of the adjoint C blocks
    size_t o_ctiles = 0;
    int32_t csplit = 1;         // RHS splits of the C blocks (1..4)
    std::vector<int4> gruns;    // runs of band tiles of the gradient's second kernel
    size_t o_gruns = 0;
    std::vector<int32_t> gorder;   // band tiles in dispatch order: by (problem, antenna block, group)
    size_t o_gorder = 0;
    std::vector<VrkLinkOut> link_host;   // output table of the link metrics, uploaded per call
    size_t o_link = 0, o_linkpart = 0;   // link-metric output table; partial sums of ||X||_F^2
    int32_t persistent = 0, grid = 0;
    int32_t max_nub = 0;
    std::vector<uint8_t> image;
    uint8_t *d_ws = nullptr;
    bool bound = false;
    // bound to the library's scratch array of device static_dev (-1: to a
    // caller workspace) by the scratch binding numbered static_gen
    int32_t static_dev = -1;
    uint64_t static_gen = 0;
};

namespace {

int32_t elem_bytes(int32_t dtype) { return dtype == VRK_C128 ? 16 : 8; }

vrk_status validate_problem(const vrk_problem &p, int idx, const vrk_options &o)
{
    if (p.nt < 1 || p.k < 1) return fail(VRK_EINVAL, "problem %d: nt=%d k=%d must be >= 1", idx, p.nt, p.k);
    if (!(p.xi > 0.0) || !std::isfinite(p.xi))
        return fail(VRK_EINVAL, "problem %d: xi=%g must be finite and > 0", idx, p.xi);
    if (!p.H || p.ldh < p.nt) return fail(VRK_EINVAL, "problem %d: H null or ldh < nt", idx);
    if (!p.vr_start || !p.vr_len) return fail(VRK_EINVAL, "problem %d: vr_start/vr_len null", idx);
    if (p.nrhs < 0) return fail(VRK_EINVAL, "problem %d: nrhs < 0", idx);
    if (p.nrhs > 0) {
        if (!p.S || p.lds < p.k) return fail(VRK_EINVAL, "problem %d: S null or lds < k", idx);
        if (!p.X || p.ldx < p.nt) return fail(VRK_EINVAL, "problem %d: X null or ldx < nt", idx);
        if (p.V && p.ldv < p.k) return fail(VRK_EINVAL, "problem %d: ldv < k", idx);
    }
    for (int i = 0; i < p.k; ++i) {
        int64_t s = p.vr_start[i], l = p.vr_len[i];
        if (s < 0 || l < 0 || s + l > p.nt)
            return fail(VRK_EINVAL, "problem %d: VR of user %d = [%lld, %lld) outside [0, %d)", idx, i,
                        (long long)s, (long long)(s + l), p.nt);
    }
    if (p.vr_mask) {
        if (p.n_sub < 1 || p.n_sub > 64 || p.nt % p.n_sub)
            return fail(VRK_EINVAL, "problem %d: n_sub=%d must be in [1, 64] and divide nt=%d", idx, p.n_sub, p.nt);
        const int32_t L = p.nt / p.n_sub;
        for (int i = 0; i < p.k; ++i) {
            const uint64_t m = p.vr_mask[i];
            if (p.n_sub < 64 && (m >> p.n_sub))
                return fail(VRK_EINVAL, "problem %d: vr_mask of user %d has bits at or above n_sub=%d", idx, i,
                            p.n_sub);
            int32_t lo = 0, hi = 0;
            if (m) {
                lo = __builtin_ctzll(m) * L;
                hi = (64 - __builtin_clzll(m)) * L;
            }
            if (p.vr_start[i] != lo || p.vr_start[i] + p.vr_len[i] != hi)
                return fail(VRK_EINVAL,
                            "problem %d: VR of user %d = [%d, %d) is not the hull [%d, %d) of its visible subarrays",
                            idx, i, p.vr_start[i], p.vr_start[i] + p.vr_len[i], lo, hi);
        }
    }
    bool any_adj = p.GX || p.GH || p.GS || p.gxi;
    if (any_adj) {
        if (!(p.GX && p.GH && p.GS && p.gxi))
            return fail(VRK_EINVAL, "problem %d: adjoint buffers GX, GH, GS, gxi must be all set or all null", idx);
        if (p.ldgx < p.nt || p.ldgh < p.nt || p.ldgs < p.k)
            return fail(VRK_EINVAL, "problem %d: adjoint strides too small", idx);
    }
    (void)o;
    return VRK_OK;
}

// Users a and b have overlapping VRs: a shared subarray under the subarray
// model, else intersecting intervals (Lemma 1: otherwise their rows are
// orthogonal).
bool vr_overlap(const ProbPlan &q, int a, int b)
{
    if (!q.mask.empty()) return (q.mask[a] & q.mask[b]) != 0;
    return std::max(q.vs[a], q.vs[b]) < std::min(q.ve[a], q.ve[b]);
}

// F on the general graph of the subarray model by reducing-peeling: while
// vertices remain, the first vertex of degree 0 joins F; else the first of
// degree 1 joins F and its neighbour is deleted; else the first vertex of
// largest degree is peeled. Peeled vertices rejoin, latest first, when no
// neighbour is in F. Degrees are kept incrementally over adjacency lists.
void build_mis_peeling(ProbPlan &q)
{
    const int K = q.p.k;
    std::vector<std::vector<int32_t>> adj(K);
    for (int a = 0; a < K; ++a)
        for (int b = a + 1; b < K; ++b)
            if (vr_overlap(q, a, b)) {
                adj[a].push_back(b);
                adj[b].push_back(a);
            }
    std::vector<int32_t> deg(K), peeled;
    std::vector<uint8_t> alive(K, 1);
    for (int v = 0; v < K; ++v) deg[v] = (int32_t)adj[v].size();
    auto remove = [&](int v) {
        alive[v] = 0;
        for (int u : adj[v])
            if (alive[u]) --deg[u];
    };
    for (int left = K; left > 0;) {
        int p0 = -1, p1 = -1, pp = -1;
        for (int v = 0; v < K; ++v) {
            if (!alive[v]) continue;
            if (deg[v] == 0 && p0 < 0) p0 = v;
            if (deg[v] == 1 && p1 < 0) p1 = v;
            if (pp < 0 || deg[v] > deg[pp]) pp = v;
        }
        if (p0 >= 0) {
            q.inf[p0] = 1;
            remove(p0);
            --left;
        } else if (p1 >= 0) {
            int w = -1;
            for (int u : adj[p1])
                if (alive[u]) w = u;
            q.inf[p1] = 1;
            remove(p1);
            remove(w);
            left -= 2;
        } else {
            peeled.push_back(pp);
            remove(pp);
            --left;
        }
    }
    for (auto it = peeled.rbegin(); it != peeled.rend(); ++it) {
        bool free_v = true;
        for (int u : adj[*it]) free_v = free_v && !q.inf[u];
        if (free_v) q.inf[*it] = 1;
    }
}

// Orthogonal set F: earliest-end greedy maximum independent set on the
// interval graph (exact there), reducing-peeling under the subarray model.
void build_mis(ProbPlan &q)
{
    const int K = q.p.k;
    q.inf.assign(K, 0);
    if (!q.mask.empty()) {
        build_mis_peeling(q);
        q.flist.clear();
        q.vlist.clear();
        for (int i = 0; i < K; ++i) (q.inf[i] ? q.flist : q.vlist).push_back(i);
        return;
    }
    std::vector<int32_t> ord;
    for (int i = 0; i < K; ++i) {
        if (q.ve[i] == q.vs[i]) q.inf[i] = 1;   // empty VR: orthogonal to every row
        else ord.push_back(i);
    }
    std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        if (q.ve[a] != q.ve[b]) return q.ve[a] < q.ve[b];
        if (q.vs[a] != q.vs[b]) return q.vs[a] < q.vs[b];
        return a < b;
    });
    int64_t last = INT64_MIN;
    for (int i : ord)
        if (q.vs[i] >= last) { q.inf[i] = 1; last = q.ve[i]; }
    q.flist.clear();
    q.vlist.clear();
    for (int i = 0; i < K; ++i) (q.inf[i] ? q.flist : q.vlist).push_back(i);
}

// Colour classes: sets of users with pairwise disjoint VRs. Interval VRs:
// optimal interval colouring (sweep by start, reuse the smallest colour whose
// interval has ended). Subarray model: greedy colouring of the mask graph,
// users in VR-start order, each taking the smallest colour none of its
// already coloured neighbours holds.
void build_colours(ProbPlan &q)
{
    const int K = q.p.k;
    q.colour.assign(K, 0);
    if (!q.mask.empty()) {
        int32_t ncol = 1;
        std::vector<uint8_t> done(K, 0), used;
        for (int i = 0; i < K; ++i) {
            const int u = q.perm[i];
            used.assign(ncol + 1, 0);
            for (int v = 0; v < K; ++v)
                if (done[v] && v != u && vr_overlap(q, u, v)) used[q.colour[v]] = 1;
            int32_t c = 0;
            while (used[c]) ++c;
            q.colour[u] = c;
            ncol = std::max(ncol, c + 1);
            done[u] = 1;
        }
        q.ncol = ncol;
    } else {
        std::vector<int32_t> ord;
        for (int i = 0; i < K; ++i)
            if (q.ve[i] > q.vs[i]) ord.push_back(i);
        std::sort(ord.begin(), ord.end(), [&](int a, int b) {
            if (q.vs[a] != q.vs[b]) return q.vs[a] < q.vs[b];
            if (q.ve[a] != q.ve[b]) return q.ve[a] < q.ve[b];
            return a < b;
        });
        using End = std::pair<int32_t, int32_t>;   // (end, colour)
        std::priority_queue<End, std::vector<End>, std::greater<End>> active;
        std::set<int32_t> freec;
        int32_t ncol = 0;
        for (int i : ord) {
            while (!active.empty() && active.top().first <= q.vs[i]) {
                freec.insert(active.top().second);
                active.pop();
            }
            int32_t c;
            if (!freec.empty()) { c = *freec.begin(); freec.erase(freec.begin()); }
            else c = ncol++;
            q.colour[i] = c;
            active.push({q.ve[i], c});
        }
        if (ncol == 0) ncol = 1;   // only empty VRs: one class
        q.ncol = ncol;
    }
    const int32_t ncol = q.ncol;
    q.col_off.assign(ncol + 1, 0);
    for (int i = 0; i < K; ++i) q.col_off[q.colour[i] + 1]++;
    for (int c = 0; c < ncol; ++c) q.col_off[c + 1] += q.col_off[c];
    q.col_users.assign(K, 0);
    std::vector<int32_t> fillp(q.col_off.begin(), q.col_off.end() - 1);
    for (int i = 0; i < K; ++i) q.col_users[fillp[q.colour[i]]++] = i;
}

void build_tables(ProbPlan &q)
{
    const vrk_problem &p = q.p;
    const int K = p.k, N = p.nt;
    q.vs.assign(p.vr_start, p.vr_start + K);
    q.ve.resize(K);
    q.mask.clear();
    q.gaps.clear();
    if (p.vr_mask) {
        q.mask.assign(p.vr_mask, p.vr_mask + K);
        const int32_t L = p.nt / p.n_sub;
        for (int u = 0; u < K; ++u) {
            const uint64_t m = q.mask[u];
            if (!m) continue;
            const int s1 = 63 - __builtin_clzll(m);
            for (int s = __builtin_ctzll(m); s <= s1;) {
                if ((m >> s) & 1u) { ++s; continue; }
                int e = s;
                while (!((m >> e) & 1u)) ++e;
                q.gaps.insert(q.gaps.end(), {u, s * L, (e - s) * L});
                s = e;
            }
        }
    }
    q.band = 0;
    for (int i = 0; i < K; ++i) { q.ve[i] = q.vs[i] + p.vr_len[i]; q.band += p.vr_len[i]; }
    // users sorted by (start, end, index)
    q.perm.resize(K);
    std::iota(q.perm.begin(), q.perm.end(), 0);
    std::sort(q.perm.begin(), q.perm.end(), [&](int a, int b) {
        if (q.vs[a] != q.vs[b]) return q.vs[a] < q.vs[b];
        if (q.ve[a] != q.ve[b]) return q.ve[a] < q.ve[b];
        return a < b;
    });
    q.pos.resize(K);
    for (int i = 0; i < K; ++i) q.pos[q.perm[i]] = i;
    // overlap sets X_k (includes k), via the sorted order
    q.xoff.assign(K + 1, 0);
    q.xidx.clear();
    for (int kk = 0; kk < K; ++kk) {
        q.xoff[kk] = (int32_t)q.xidx.size();
        for (int j = 0; j < K; ++j)
            if (j == kk || vr_overlap(q, kk, j)) q.xidx.push_back(j);
    }
    q.xoff[K] = (int32_t)q.xidx.size();
    build_mis(q);
    build_colours(q);
    q.fch.clear();
    for (int f : q.flist) q.fch.push_back(q.pos[f] / 4);
    std::sort(q.fch.begin(), q.fch.end());
    q.fch.erase(std::unique(q.fch.begin(), q.fch.end()), q.fch.end());
    // gather lists: users meeting each 64-antenna block
    const int ngb = (N + VRK_GATHER_BLOCK - 1) / VRK_GATHER_BLOCK;
    q.gb_off.assign(ngb + 1, 0);
    q.gb_users.clear();
    for (int g = 0; g < ngb; ++g) {
        q.gb_off[g] = (int32_t)q.gb_users.size();
        int32_t lo = g * VRK_GATHER_BLOCK, hi = std::min(N, lo + VRK_GATHER_BLOCK);
        for (int i = 0; i < K; ++i)
            if (std::max(lo, q.vs[i]) < std::min(hi, q.ve[i])) q.gb_users.push_back(i);
    }
    q.gb_off[ngb] = (int32_t)q.gb_users.size();
    // MFMA tiles (sorted user order)
    q.nub = (K + VRK_UB - 1) / VRK_UB;
    q.nab = (N + VRK_AB - 1) / VRK_AB;
    q.ntile = (p.nrhs + VRK_TILE_RHS - 1) / VRK_TILE_RHS;
    q.rab_lo.assign(q.nub, 0);
    q.rab_hi.assign(q.nub, 0);
    q.ha_off.assign(q.nub + 1, 0);
    for (int ub = 0; ub < q.nub; ++ub) {
        int32_t lo = INT32_MAX, hi = INT32_MIN;
        for (int i = ub * VRK_UB; i < std::min(K, (ub + 1) * VRK_UB); ++i) {
            int u = q.perm[i];
            if (q.ve[u] == q.vs[u]) continue;
            lo = std::min(lo, q.vs[u] / VRK_AB);
            hi = std::max(hi, (q.ve[u] + VRK_AB - 1) / VRK_AB);
        }
        if (lo > hi) lo = hi = 0;
        q.rab_lo[ub] = lo;
        q.rab_hi[ub] = hi;
        q.ha_off[ub + 1] = q.ha_off[ub] + 4 * (int64_t)(hi - lo);
    }
    q.n_ha = q.ha_off[q.nub];
    const int nuc = q.nub * (VRK_UB / 4);
    q.ag_off.assign(q.nab + 1, 0);
    q.ag_uc.clear();
    for (int ab = 0; ab < q.nab; ++ab) {
        q.ag_off[ab] = (int32_t)q.ag_uc.size();
        int32_t lo = ab * VRK_AB, hi = lo + VRK_AB;
        for (int uc = 0; uc < nuc; ++uc) {
            bool any = false;
            for (int t = 0; t < 4; ++t) {
                int i = uc * 4 + t;
                if (i >= K) break;
                int u = q.perm[i];
                if (std::max(lo, q.vs[u]) < std::min(hi, q.ve[u])) any = true;
            }
            if (any) q.ag_uc.push_back(uc);
        }
    }
    q.ag_off[q.nab] = (int32_t)q.ag_uc.size();
    q.n_hg = (int64_t)q.ag_uc.size();
    // Gram blocks (16-user block, 4-user chunk) with any pair of overlapping
    // VRs (a shared subarray under the subarray model) or a shared user (the diagonal), in VR-start order. Per block the
    // chunks holding a user of F come first, so the orthogonal half-step
    // (phi nonzero on F only) needs only the groups covering the first
    // gm_nf entries; the list is padded to groups of 4 chunks, loaded and
    // multiplied at once (padding chunks, -1, hold zero tiles).
    q.gm_off.assign(q.nub + 1, 0);
    q.gm_nf.assign(q.nub, 0);
    q.gm_c.clear();
    for (int mb = 0; mb < q.nub; ++mb) {
        q.gm_off[mb] = (int32_t)q.gm_c.size();
        std::vector<int32_t> with_f, rest;
        for (int uc = 0; uc < nuc; ++uc) {
            bool any = false, hasf = false;
            for (int t = 0; t < 4; ++t)
                if (uc * 4 + t < K && q.inf[q.perm[uc * 4 + t]]) hasf = true;
            for (int i = mb * VRK_UB; i < std::min(K, (mb + 1) * VRK_UB) && !any; ++i)
                for (int t = 0; t < 4 && !any; ++t) {
                    const int kv = uc * 4 + t;
                    if (kv >= K) break;
                    const int a = q.perm[i], b = q.perm[kv];
                    any = (a == b) || vr_overlap(q, a, b);
                }
            if (any) (hasf ? with_f : rest).push_back(uc);
        }
        q.gm_nf[mb] = (int32_t)with_f.size();
        q.gm_c.insert(q.gm_c.end(), with_f.begin(), with_f.end());
        q.gm_c.insert(q.gm_c.end(), rest.begin(), rest.end());
        while ((q.gm_c.size() - q.gm_off[mb]) % 4) q.gm_c.push_back(-1);
    }
    q.gm_off[q.nub] = (int32_t)q.gm_c.size();
    q.n_gm = (int64_t)q.gm_c.size();
    q.gm_fs.assign(q.gm_c.size(), VRK_WAVE_FCHUNKS);
    for (size_t e = 0; e < q.gm_c.size(); ++e) {
        const auto it = std::lower_bound(q.fch.begin(), q.fch.end(), q.gm_c[e]);
        if (q.gm_c[e] >= 0 && it != q.fch.end() && *it == q.gm_c[e] && it - q.fch.begin() < VRK_WAVE_FCHUNKS)
            q.gm_fs[e] = (int32_t)(it - q.fch.begin());
    }
    // 16 x 16 blocks (ub, ub') of the same pattern, for C = sum_b v_b mu_b^H
    // of the adjoint gradient; the pattern is symmetric and holds every
    // diagonal block
    q.cp_off.assign(q.nub + 1, 0);
    q.cp_col.clear();
    for (int mb = 0; mb < q.nub; ++mb) {
        q.cp_off[mb] = (int32_t)q.cp_col.size();
        std::vector<int32_t> cols;
        for (int e = q.gm_off[mb]; e < q.gm_off[mb + 1]; ++e)
            if (q.gm_c[e] >= 0) cols.push_back(q.gm_c[e] / (VRK_UB / 4));
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        q.cp_col.insert(q.cp_col.end(), cols.begin(), cols.end());
    }
    q.cp_off[q.nub] = (int32_t)q.cp_col.size();
    auto find_block = [&](int r, int c) {
        auto b0 = q.cp_col.begin() + q.cp_off[r], b1 = q.cp_col.begin() + q.cp_off[r + 1];
        auto it = std::lower_bound(b0, b1, c);
        return (it != b1 && *it == c) ? (int32_t)(it - q.cp_col.begin()) : -1;
    };
    q.cp_tr.assign(q.cp_col.size(), -1);
    q.cp_diag.assign(q.nub, -1);
    for (int mb = 0; mb < q.nub; ++mb) {
        for (int e = q.cp_off[mb]; e < q.cp_off[mb + 1]; ++e) q.cp_tr[e] = find_block(q.cp_col[e], mb);
        q.cp_diag[mb] = find_block(mb, mb);
    }
}

template <class T>
void put(std::vector<uint8_t> &img, size_t off, const std::vector<T> &v)
{
    if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(T));
}

}  // namespace

extern "C" {

void vrk_default_options(vrk_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->variant = VRK_VR_OAHK;
    o->select = VRK_SEL_BAIWU;
    o->dtype = VRK_C64;
    o->engine = VRK_ENGINE_AUTO;
    o->tol = 1e-5;
    o->max_iters = 100000;
    o->seed = 0;
    o->schedule = VRK_SCHED_AUTO;
    o->tile_waves = 0;
    o->persistent = 0;
    o->wave_tiles = 0;
    o->check_every = 1;
}

vrk_status vrk_plan_create(const vrk_problem *probs, int32_t nprob, const vrk_options *opt,
                           size_t *ws_bytes, vrk_plan **out)
{
    g_err.clear();
    if (!out || !ws_bytes) return fail(VRK_EINVAL, "out and ws_bytes must be non-null");
    *out = nullptr;
    if (!probs || nprob < 1) return fail(VRK_EINVAL, "need at least one problem");
    if (!opt) return fail(VRK_EINVAL, "options null");
    const vrk_options &o = *opt;
    if (o.variant < 0 || o.variant > 3) return fail(VRK_EINVAL, "variant %d", o.variant);
    if (o.select < 0 || o.select > 4) return fail(VRK_EINVAL, "select %d", o.select);
    if (o.dtype != VRK_C64 && o.dtype != VRK_C128) return fail(VRK_EINVAL, "dtype %d", o.dtype);
    if (o.engine < 0 || o.engine > 2) return fail(VRK_EINVAL, "engine %d", o.engine);
    if (o.schedule < 0 || o.schedule > 2) return fail(VRK_EINVAL, "schedule %d", o.schedule);
    if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return fail(VRK_EINVAL, "tol %g", o.tol);
    if (o.max_iters < 1) return fail(VRK_EINVAL, "max_iters must be >= 1");
    if (o.check_every < 0) return fail(VRK_EINVAL, "check_every must be >= 0 (0: every iteration)");
    if (o.tile_waves != 0 && o.tile_waves != 1 && o.tile_waves != 4 && o.tile_waves != 8 && o.tile_waves != 16)
        return fail(VRK_EINVAL, "tile_waves %d", o.tile_waves);
    if (o.wave_tiles != -1 && o.wave_tiles != 0 && o.wave_tiles != 1 && o.wave_tiles != 2 && o.wave_tiles != 4 &&
        o.wave_tiles != 8)
        return fail(VRK_EINVAL, "wave_tiles %d", o.wave_tiles);
    for (int i = 0; i < nprob; ++i) {
        vrk_status s = validate_problem(probs[i], i, o);
        if (s != VRK_OK) return s;
    }
    vrk_plan *pl = new vrk_plan();
    pl->opt = o;
    pl->pp.resize(nprob);
    bool all_adj = true;
    int32_t max_nt = 0, max_k = 0, min_rhs = INT32_MAX, max_kpad = 0;
    for (int i = 0; i < nprob; ++i) {
        ProbPlan &q = pl->pp[i];
        q.p = probs[i];
        build_tables(q);
        q.rhs_base = pl->total_rhs;
        pl->total_rhs += q.p.nrhs;
        pl->max_rhs = std::max(pl->max_rhs, q.p.nrhs);
        pl->max_k = std::max(pl->max_k, q.p.k);
        all_adj = all_adj && q.p.GX;
        pl->any_gaps = pl->any_gaps || !q.gaps.empty();
        max_nt = std::max(max_nt, q.p.nt);
        max_k = std::max(max_k, q.p.k);
        max_kpad = std::max(max_kpad, q.nub * VRK_UB);
        min_rhs = std::min(min_rhs, q.p.nrhs);
        q.p.vr_start = nullptr;   // the caller's host arrays are not kept
        q.p.vr_len = nullptr;
        q.p.vr_mask = nullptr;
    }
    pl->adjoint_ready = all_adj;
    // engine choice
    int32_t waves = o.tile_waves ? o.tile_waves : 16;   // four waves per SIMD by default
    bool mfma_ok = o.dtype == VRK_C64 && vrk_mfma_supported(max_kpad, waves);
    int32_t eng = o.engine;
    if (eng == VRK_ENGINE_AUTO) eng = (mfma_ok && min_rhs >= VRK_TILE_RHS) ? VRK_ENGINE_MFMA : VRK_ENGINE_VECTOR;
    if (eng == VRK_ENGINE_MFMA && !mfma_ok) {
        delete pl;
        return fail(VRK_EUNSUPPORTED, "MFMA engine needs complex64, 8 or 16 waves and k <= %d with %d waves",
                    16 * waves, waves);
    }
    pl->engine = eng;
    pl->waves = waves;
    pl->schedule = o.schedule == VRK_SCHED_AUTO ? VRK_SCHED_GATHER : o.schedule;
    pl->max_nt = max_nt;
    bool any_masked = false;
    for (auto &q : pl->pp) any_masked = any_masked || !q.mask.empty();
    // small-channel form of the vector engine (the channel zero-padded in
    // LDS, x in registers, a wave per 64-antenna slot up to four): forced by
    // tile_waves 1, the general form by 4, else chosen whenever it fits
    const bool small_ok = eng == VRK_ENGINE_VECTOR && vrk_small_supported(o.dtype, max_nt, max_k, any_masked ? 1 : 0);
    if (eng == VRK_ENGINE_VECTOR && o.tile_waves == 1 && !small_ok) {
        delete pl;
        return fail(VRK_EUNSUPPORTED,
                    "small-channel vector engine needs nt <= 1024, k <= 64, interval VRs and the channel, "
                    "zero-padded to 16-row blocks of 64, 128, 256, 512 or 1024 antennas, within 128 KiB "
                    "(nt %d, k %d)",
                    max_nt, max_k);
    }
    if (small_ok && o.tile_waves != 4) {
        pl->small = true;
        pl->waves = 1;
        pl->lds = vrk_small_lds_bytes(o.dtype, max_nt, max_k);
    } else if (eng == VRK_ENGINE_VECTOR) {
        pl->waves = 4;
        pl->lds = vrk_vec_lds_bytes(o.dtype, max_nt, max_k);
        if (pl->lds > 160 * 1024) {
            delete pl;
            return fail(VRK_EUNSUPPORTED, "vector engine needs %zu bytes of LDS (> 160 KiB) for nt=%d k=%d",
                        pl->lds, max_nt, max_k);
        }
        // small channels: the workgroup keeps H (K x Nt) and the plan tables
        // its steps read in LDS after its state, so the iterations wait on no
        // memory; the whole allocation stays within 96 KiB
        size_t extra = 0;
        for (auto &q : pl->pp) {
            const size_t tb = 4 * (2 * (size_t)q.p.k + q.flist.size() + q.vlist.size() + q.gb_off.size() +
                                   q.gb_users.size() + q.xoff.size() + q.xidx.size()) +
                              (size_t)q.p.k;
            const size_t hb = 16 + (size_t)q.p.k * q.p.nt * elem_bytes(o.dtype) + tb;
            q.stage_h = pl->lds + hb <= 96 * 1024;
            if (q.stage_h) extra = std::max(extra, hb);
        }
        pl->lds += extra;
    } else {
        int32_t max_nab = (max_nt + VRK_AB - 1) / VRK_AB;
        pl->ep = vrk_mfma_entries(max_kpad, waves);
        const bool greedy = o.variant == VRK_GRK || o.variant == VRK_VR_OGRK;
        // VR-OAHK with few users in F and a nonempty V takes the orthogonal
        // half-step on the VALU from the F columns of M (held in LDS), unless
        // each thread holds four entries (then it stays on the MFMA)
        int32_t max_nmf = 0;
        for (auto &q : pl->pp) {
            q.nmf = 0;
            q.fpos.clear();
            const int nf = (int)q.flist.size();
            if (o.variant == VRK_VR_OAHK && nf >= 1 && nf <= 16 && !q.vlist.empty() && pl->ep < 4) {
                q.nmf = nf;
                for (int f : q.flist) q.fpos.push_back(q.pos[f]);
            }
            max_nmf = std::max(max_nmf, q.nmf);
        }
        pl->lds = vrk_mfma_lds_bytes(max_kpad, max_nab, waves, greedy ? 1 : 0, max_nmf);
        if (pl->lds > 160 * 1024) {
            delete pl;
            return fail(VRK_EUNSUPPORTED, "MFMA engine needs %zu bytes of LDS for k=%d", pl->lds, max_k);
        }
        pl->waves_adj = waves;
        pl->ep_adj = pl->ep;
        pl->lds_adj = pl->lds;
        if (o.tile_waves == 0 && all_adj && max_kpad <= 64 && vrk_mfma_supported(max_kpad, 8)) {
            // with few users the adjoint solve runs faster on 8-wave tiles
            // (measured on 64 users: 5 us of 83), the forward one on 16
            const size_t l8 = vrk_mfma_lds_bytes(max_kpad, max_nab, 8, greedy ? 1 : 0, max_nmf);
            if (l8 <= 160 * 1024) {
                pl->waves_adj = 8;
                pl->ep_adj = vrk_mfma_entries(max_kpad, 8);
                pl->lds_adj = l8;
            }
        }
        // Wave-owned tiles for the aggregated sweeps: forced by wave_tiles > 0,
        // or chosen when the batch is many tiles deep (several tiles per
        // compute unit) and the block tiles are not asked for
        {
            int64_t ntiles = 0;
            size_t max_fch = 0;
            for (auto &q : pl->pp) {
                ntiles += q.ntile;
                max_fch = std::max(max_fch, q.fch.size());
            }
            const bool agg = o.variant == VRK_AHK || o.variant == VRK_VR_OAHK;
            const bool fits = o.variant != VRK_VR_OAHK || max_fch <= VRK_WAVE_FCHUNKS;
            int32_t T = 0;
            if (o.wave_tiles > 0) {
                if (!agg || !fits || o.persistent) {
                    delete pl;
                    return fail(VRK_EUNSUPPORTED,
                                "wave-owned tiles need AHK or VR-OAHK, at most %d chunks of F users per drop "
                                "(here %zu) and no persistent launch", VRK_WAVE_FCHUNKS, max_fch);
                }
                T = o.wave_tiles;
            } else if (o.wave_tiles == 0 && agg && fits && o.tile_waves == 0 && !o.persistent) {
                // two row blocks per wave (the 128-register build: four waves
                // per SIMD), so the waves per tile follow K; taken when the
                // batch has enough tiles for about four waves per SIMD
                const int32_t nubm = max_kpad / VRK_UB;
                int32_t t = 1;
                while (2 * t < nubm) t *= 2;
                if (ntiles * t >= 4096) T = t;
            }
            if (T > 0) {
                const int32_t nubm = max_kpad / VRK_UB;
                const int32_t bpw = (nubm + T - 1) / T <= 2 ? 2 : 4;
                if (!vrk_wave_supported(o.variant, max_kpad, T, bpw)) {
                    delete pl;
                    return fail(VRK_EUNSUPPORTED, "wave-owned tiles: %d waves cannot own %d row blocks", T, nubm);
                }
                pl->wave_T = T;
                pl->wave_bpw = bpw;
                pl->lds_wave = vrk_wave_lds_bytes(o.variant, max_kpad, T);
                if (pl->lds_wave > 160 * 1024) {
                    delete pl;
                    return fail(VRK_EUNSUPPORTED, "wave-owned tiles need %zu bytes of LDS", pl->lds_wave);
                }
            }
        }
        // Work items (problem, tile). Problems go to the XCD queues by cost,
        // largest first onto the least loaded queue, so each XCD's L2 holds
        // few channels at a time; within a queue the most expensive tiles
        // come first.
        std::vector<int> order(nprob);
        std::iota(order.begin(), order.end(), 0);
        auto cost = [&](int i) { return (double)(pl->pp[i].n_ha + pl->pp[i].n_hg) * pl->pp[i].ntile; };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
        std::vector<std::vector<int>> qprobs(VRK_NQUEUE);
        double load[VRK_NQUEUE] = {0};
        for (int i : order) {
            int qi = (int)(std::min_element(load, load + VRK_NQUEUE) - load);
            qprobs[qi].push_back(i);
            load[qi] += cost(i);
        }
        for (int qi = 0; qi < VRK_NQUEUE; ++qi) {
            pl->qbase[qi] = (int32_t)pl->work.size();
            for (int i : qprobs[qi])
                for (int t = 0; t < pl->pp[i].ntile; ++t) pl->work.push_back({i, t});
            pl->qsize[qi] = (int32_t)pl->work.size() - pl->qbase[qi];
        }
        pl->persistent = o.persistent ? 1 : 0;
        for (int i = 0; i < nprob; ++i) pl->max_nub = std::max(pl->max_nub, pl->pp[i].nub);
        if (all_adj)
            for (int i = 0; i < nprob; ++i) {
                const ProbPlan &q = pl->pp[i];
                // (problem, user-block group, antenna block, flags) for every
                // antenna block that some block of the group meets; flags: 1 on
                // the problem's first tile, which also carries its tile count
                int first = 1;
                const size_t t0 = pl->gtiles.size();
                for (int ubg = 0; ubg * VRK_GRAD_UG < q.nub; ++ubg) {
                    const int u0 = ubg * VRK_GRAD_UG, u1 = std::min(q.nub, u0 + VRK_GRAD_UG);
                    for (int ab = 0; ab < q.nab; ++ab) {
                        bool meets = false;
                        for (int ub = u0; ub < u1; ++ub) meets = meets || (q.rab_lo[ub] <= ab && ab < q.rab_hi[ub]);
                        if (!meets) continue;
                        pl->gtiles.push_back(make_int4(i, ubg, ab, first));
                        first = 0;
                    }
                }
                if (first) pl->gtiles.push_back(make_int4(i, -1, 0, 1));
                pl->gtiles[t0].w |= (int32_t)(pl->gtiles.size() - t0) << 2;
            }
        if (!pl->gtiles.empty()) {
            // enough 4-wave workgroups to fill the device (about 4096), each
            // split keeping at least 64 right-hand sides (16 per wave)
            int64_t want = 4096 / (int64_t)pl->gtiles.size();
            int64_t cap = std::max<int64_t>(1, min_rhs / 64);
            pl->gsplit = (int32_t)std::max<int64_t>(1, std::min<int64_t>({want, cap, 16}));
            // C blocks: up to 4 RHS splits while there are fewer than 1024
            // blocks, each split keeping at least 256 right-hand sides
            int64_t nblk = 0;
            for (const auto &q : pl->pp) nblk += (int64_t)q.cp_col.size();
            pl->csplit = (int32_t)std::max<int64_t>(
                1, std::min<int64_t>({1024 / std::max<int64_t>(1, nblk), min_rhs / 256, 4}));
            for (int i = 0; i < nprob; ++i) {
                const ProbPlan &q = pl->pp[i];
                for (int mb = 0; mb < q.nub; ++mb)
                    for (int e = q.cp_off[mb]; e < q.cp_off[mb + 1]; ++e)
                        for (int cs = 0; cs < pl->csplit; ++cs) pl->ctiles.push_back(make_int4(i, e, cs, mb));
            }
            // dispatch order of the band tiles: the groups that meet one
            // antenna block next to each other, so that they read its columns
            // of the incoming gradient from one XCD's L2 at about one time
            pl->gorder.resize(pl->gtiles.size());
            for (size_t t = 0; t < pl->gtiles.size(); ++t) pl->gorder[t] = (int32_t)t;
            std::stable_sort(pl->gorder.begin(), pl->gorder.end(), [&](int32_t a, int32_t b) {
                const int4 &ta = pl->gtiles[a], &tb = pl->gtiles[b];
                if (ta.x != tb.x) return ta.x < tb.x;
                return ta.z < tb.z;
            });
            // runs of at most R consecutive band tiles of one (problem, user
            // block group), R chosen for about 1024 runs
            const int R = (int)std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)pl->gtiles.size() / 1024));
            for (size_t t = 0; t < pl->gtiles.size();) {
                const int4 a = pl->gtiles[t];
                size_t e = t + 1;
                while (e < pl->gtiles.size() && e - t < (size_t)R && pl->gtiles[e].x == a.x && pl->gtiles[e].y == a.y)
                    ++e;
                const bool first = t == 0 || pl->gtiles[t - 1].x != a.x;
                pl->gruns.push_back(make_int4((int32_t)t, (int32_t)(e - t), first ? 1 : 0, 0));
                t = e;
            }
        }
    }
    // workspace carving
    const int32_t eb = elem_bytes(o.dtype), rb = o.dtype == VRK_C128 ? 8 : 4;
    Carver cv;
    pl->o_desc = cv.take(sizeof(VrkDesc) * nprob);
    pl->o_work = cv.take(sizeof(VrkWork) * std::max<size_t>(1, pl->work.size()));
    pl->o_gtiles = cv.take(sizeof(int4) * std::max<size_t>(1, pl->gtiles.size()));
    pl->o_queue = cv.take(sizeof(int32_t) * 3 * VRK_NQUEUE);
    pl->o_ctiles = cv.take(sizeof(int4) * std::max<size_t>(1, pl->ctiles.size()));
    pl->o_gruns = cv.take(sizeof(int4) * std::max<size_t>(1, pl->gruns.size()));
    pl->o_gorder = cv.take(sizeof(int32_t) * std::max<size_t>(1, pl->gorder.size()));
    for (auto &q : pl->pp) {
        const int K = q.p.k;
        q.o_vs = cv.take(4 * K);
        q.o_ve = cv.take(4 * K);
        q.o_xoff = cv.take(4 * (K + 1));
        q.o_xidx = cv.take(4 * q.xidx.size());
        q.o_flist = cv.take(4 * q.flist.size());
        q.o_vlist = cv.take(4 * q.vlist.size());
        q.o_inf = cv.take(K);
        q.o_coloff = cv.take(4 * q.col_off.size());
        q.o_colusr = cv.take(4 * q.col_users.size());
        q.o_gboff = cv.take(4 * q.gb_off.size());
        q.o_gbusr = cv.take(4 * q.gb_users.size());
        q.o_perm = cv.take(4 * K);
        q.o_pos = cv.take(4 * K);
        q.o_rablo = cv.take(4 * q.rab_lo.size());
        q.o_rabhi = cv.take(4 * q.rab_hi.size());
        q.o_haoff = cv.take(8 * q.ha_off.size());
        q.o_agoff = cv.take(4 * q.ag_off.size());
        q.o_aguc = cv.take(4 * q.ag_uc.size());
        q.o_gmoff = cv.take(4 * q.gm_off.size());
        q.o_gmc = cv.take(4 * q.gm_c.size());
        q.o_gmnf = cv.take(4 * q.gm_nf.size());
        q.o_fpos = cv.take(4 * q.fpos.size());
        q.o_cpoff = cv.take(4 * q.cp_off.size());
        q.o_cpcol = cv.take(4 * q.cp_col.size());
        q.o_cptr = cv.take(4 * q.cp_tr.size());
        q.o_cpdiag = cv.take(4 * q.cp_diag.size());
        q.o_gaps = cv.take(4 * q.gaps.size());
        q.o_mask = cv.take(8 * q.mask.size());
        q.o_fch = cv.take(4 * q.fch.size());
        q.o_gmfs = cv.take(4 * q.gm_fs.size());
    }
    pl->table_end = cv.off;
    pl->o_link = cv.take(sizeof(VrkLinkOut) * nprob);
    pl->o_linkpart = cv.take(sizeof(double) * VRK_LINK_GROUPS * nprob);
    pl->o_gpart = cv.take(pl->gsplit > 1 ? pl->gtiles.size() * (size_t)pl->gsplit * VRK_GRAD_UG * 256 * 8 : 0);
    for (auto &q : pl->pp) {
        q.o_nrm = cv.take((size_t)rb * std::max(q.p.k, q.nub * VRK_UB));
        q.o_fro2 = cv.take(rb);
        if (eng == VRK_ENGINE_MFMA) {
            q.o_ha = cv.take(q.n_ha * 64 * 8);
            q.o_hg = cv.take(q.n_hg * 64 * 8);
            q.o_gm = cv.take(q.n_gm * 64 * 8);
            q.o_mf = cv.take((size_t)q.nub * VRK_UB * q.nmf * 8);
            pl->max_tiles = std::max(pl->max_tiles, q.n_gm);
            pl->max_tiles = std::max(pl->max_tiles, (int64_t)(q.nub * VRK_UB * q.nmf + 63) / 64);
            pl->max_tiles = std::max(pl->max_tiles, std::max(q.n_ha, q.n_hg));
        }
        // v of the forward solve is kept when the caller passes no V: the
        // adjoint needs it, and so do the link metrics of an S = I_K solve
        // (E = (M - xi I) V^T on the matrix cores)
        q.keep_v = !q.p.V && (q.p.GX || q.p.nrhs == q.p.k);
        q.o_vfwd = q.keep_v ? cv.take((size_t)eb * q.p.nrhs * q.p.k) : 0;
        if (q.p.GX) {
            q.o_sadj = cv.take((size_t)eb * q.p.nrhs * q.p.k);
            q.o_xadj = eng == VRK_ENGINE_MFMA ? 0 : cv.take((size_t)eb * q.p.nrhs * q.p.nt);
            if (eng == VRK_ENGINE_MFMA) {
                q.o_vsrt = cv.take((size_t)8 * q.p.nrhs * q.nub * VRK_UB);
                q.o_msrt = cv.take((size_t)8 * q.p.nrhs * q.nub * VRK_UB);
                q.o_cblk = cv.take((size_t)8 * 256 * q.cp_col.size() * pl->csplit);
            }
        }
    }
    pl->ws_bytes = cv.off;
    *ws_bytes = pl->ws_bytes;
    *out = pl;
    return VRK_OK;
}

}  // extern "C"

// The kernels that read H: row norms and ||A||_F^2, and on the MFMA engine
// the residual, aggregation and Gram tiles (with the F columns of M).
static vrk_status channel_kernels(vrk_plan *pl, uint8_t *base, hipStream_t s)
{
    const VrkDesc *dd = reinterpret_cast<const VrkDesc *>(base + pl->o_desc);
    hipError_t e = vrk_launch_norms(dd, (int32_t)pl->pp.size(), pl->opt.dtype, s);
    if (e != hipSuccess) return hip_fail(e, "row-norm kernel");
    if (pl->engine == VRK_ENGINE_MFMA) {
        e = vrk_launch_pack(dd, (int32_t)pl->pp.size(), pl->max_tiles, s);
        if (e != hipSuccess) return hip_fail(e, "tile-pack kernel");
    }
    return VRK_OK;
}

// Tables into the workspace at d_ws (checked by the caller), then the
// row-norm and tile kernels; shared by both binding entry points.
static vrk_status bind_at(vrk_plan *pl, void *d_ws, void *stream)
{
    pl->bound = false;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *base = reinterpret_cast<uint8_t *>(d_ws);
    pl->image.assign(pl->table_end, 0);
    pl->link_host.clear();   // the link-metric output table is not in this workspace yet
    std::vector<VrkDesc> descs(pl->pp.size());
    const vrk_options &o = pl->opt;
    const int32_t eb = elem_bytes(o.dtype);
    for (size_t i = 0; i < pl->pp.size(); ++i) {
        ProbPlan &q = pl->pp[i];
        auto &img = pl->image;
        put(img, q.o_vs, q.vs);
        put(img, q.o_ve, q.ve);
        put(img, q.o_xoff, q.xoff);
        put(img, q.o_xidx, q.xidx);
        put(img, q.o_flist, q.flist);
        put(img, q.o_vlist, q.vlist);
        put(img, q.o_inf, q.inf);
        put(img, q.o_coloff, q.col_off);
        put(img, q.o_colusr, q.col_users);
        put(img, q.o_gboff, q.gb_off);
        put(img, q.o_gbusr, q.gb_users);
        put(img, q.o_perm, q.perm);
        put(img, q.o_pos, q.pos);
        put(img, q.o_rablo, q.rab_lo);
        put(img, q.o_rabhi, q.rab_hi);
        put(img, q.o_haoff, q.ha_off);
        put(img, q.o_agoff, q.ag_off);
        put(img, q.o_aguc, q.ag_uc);
        put(img, q.o_gmoff, q.gm_off);
        put(img, q.o_gmc, q.gm_c);
        put(img, q.o_gmnf, q.gm_nf);
        put(img, q.o_cpoff, q.cp_off);
        put(img, q.o_cpcol, q.cp_col);
        put(img, q.o_cptr, q.cp_tr);
        put(img, q.o_cpdiag, q.cp_diag);
        put(img, q.o_fpos, q.fpos);
        put(img, q.o_gaps, q.gaps);
        put(img, q.o_mask, q.mask);
        put(img, q.o_fch, q.fch);
        put(img, q.o_gmfs, q.gm_fs);
        VrkDesc &d = descs[i];
        std::memset(&d, 0, sizeof d);
        const vrk_problem &p = q.p;
        d.nt = p.nt; d.k = p.k; d.nrhs = p.nrhs;
        d.nf = (int32_t)q.flist.size(); d.nv = (int32_t)q.vlist.size();
        d.ncol = q.ncol; d.ngb = (int32_t)q.gb_off.size() - 1; d.nub = q.nub;
        d.nab = q.nab; d.ntile = q.ntile;
        d.xi = p.xi;
        d.ldh = p.ldh; d.lds = p.lds; d.ldx = p.ldx; d.ldv = p.V ? p.ldv : p.k;
        d.ldgx = p.ldgx; d.ldgh = p.ldgh; d.ldgs = p.ldgs;
        d.rhs_base = q.rhs_base;
        d.H = p.H; d.S = p.S; d.X = p.X;
        d.V = p.V ? p.V : (q.keep_v ? base + q.o_vfwd : nullptr);
        d.GX = p.GX; d.GH = p.GH; d.GS = p.GS; d.gxi = p.gxi;
        d.Sadj = p.GX ? base + q.o_sadj : nullptr;
        d.Xadj = p.GX && pl->engine != VRK_ENGINE_MFMA ? base + q.o_xadj : nullptr;
        d.Vfwd = nullptr;
        const bool srt = p.GX && pl->engine == VRK_ENGINE_MFMA;
        d.Vsrt = srt ? base + q.o_vsrt : nullptr;
        d.Msrt = srt ? base + q.o_msrt : nullptr;
        d.cp_off = (const int32_t *)(base + q.o_cpoff);
        d.cp_col = (const int32_t *)(base + q.o_cpcol);
        d.cp_tr = (const int32_t *)(base + q.o_cptr);
        d.cp_diag = (const int32_t *)(base + q.o_cpdiag);
        d.Cblk = srt ? base + q.o_cblk : nullptr;
        d.vs = (const int32_t *)(base + q.o_vs);
        d.ve = (const int32_t *)(base + q.o_ve);
        d.xoff = (const int32_t *)(base + q.o_xoff);
        d.xidx = (const int32_t *)(base + q.o_xidx);
        d.flist = (const int32_t *)(base + q.o_flist);
        d.vlist = (const int32_t *)(base + q.o_vlist);
        d.inf = (const uint8_t *)(base + q.o_inf);
        d.col_off = (const int32_t *)(base + q.o_coloff);
        d.col_users = (const int32_t *)(base + q.o_colusr);
        d.gb_off = (const int32_t *)(base + q.o_gboff);
        d.gb_users = (const int32_t *)(base + q.o_gbusr);
        d.perm = (const int32_t *)(base + q.o_perm);
        d.pos = (const int32_t *)(base + q.o_pos);
        d.nrm = base + q.o_nrm;
        d.fro2 = base + q.o_fro2;
        d.rab_lo = (const int32_t *)(base + q.o_rablo);
        d.rab_hi = (const int32_t *)(base + q.o_rabhi);
        d.ha_off = (const int64_t *)(base + q.o_haoff);
        d.ag_off = (const int32_t *)(base + q.o_agoff);
        d.ag_uc = (const int32_t *)(base + q.o_aguc);
        d.HA = pl->engine == VRK_ENGINE_MFMA ? base + q.o_ha : nullptr;
        d.HG = pl->engine == VRK_ENGINE_MFMA ? base + q.o_hg : nullptr;
        d.gm_off = (const int32_t *)(base + q.o_gmoff);
        d.gm_c = (const int32_t *)(base + q.o_gmc);
        d.gm_nf = (const int32_t *)(base + q.o_gmnf);
        d.GM = pl->engine == VRK_ENGINE_MFMA ? base + q.o_gm : nullptr;
        d.nmf = pl->engine == VRK_ENGINE_MFMA ? q.nmf : 0;
        d.MF = d.nmf ? base + q.o_mf : nullptr;
        d.fpos = (const int32_t *)(base + q.o_fpos);
        d.masked = q.mask.empty() ? 0 : 1;
        d.stage_h = (pl->engine == VRK_ENGINE_VECTOR && q.stage_h) ? 1 : 0;
        d.sub_len = q.mask.empty() ? 0 : p.nt / p.n_sub;
        d.vmask = (const uint64_t *)(base + q.o_mask);
        d.ngap = (int32_t)(q.gaps.size() / 3);
        d.gaps = (const int32_t *)(base + q.o_gaps);
        d.nfch = (int32_t)q.fch.size();
        d.fch = (const int32_t *)(base + q.o_fch);
        d.gm_fs = (const int32_t *)(base + q.o_gmfs);
        (void)eb;
    }
    std::memcpy(pl->image.data() + pl->o_desc, descs.data(), sizeof(VrkDesc) * descs.size());
    if (!pl->work.empty())
        std::memcpy(pl->image.data() + pl->o_work, pl->work.data(), sizeof(VrkWork) * pl->work.size());
    if (!pl->gtiles.empty())
        std::memcpy(pl->image.data() + pl->o_gtiles, pl->gtiles.data(), sizeof(int4) * pl->gtiles.size());
    if (!pl->ctiles.empty())
        std::memcpy(pl->image.data() + pl->o_ctiles, pl->ctiles.data(), sizeof(int4) * pl->ctiles.size());
    if (!pl->gruns.empty())
        std::memcpy(pl->image.data() + pl->o_gruns, pl->gruns.data(), sizeof(int4) * pl->gruns.size());
    if (!pl->gorder.empty())
        std::memcpy(pl->image.data() + pl->o_gorder, pl->gorder.data(), sizeof(int32_t) * pl->gorder.size());
    {
        int32_t *qv = reinterpret_cast<int32_t *>(pl->image.data() + pl->o_queue);
        for (int qi = 0; qi < VRK_NQUEUE; ++qi) {
            qv[qi] = 0;
            qv[VRK_NQUEUE + qi] = pl->qbase[qi];
            qv[2 * VRK_NQUEUE + qi] = pl->qsize[qi];
        }
    }
    hipError_t e = hipMemcpyAsync(base, pl->image.data(), pl->table_end, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(plan tables)");
    if (vrk_status st = channel_kernels(pl, base, s)) return st;
    if (pl->engine == VRK_ENGINE_MFMA) {
        VrkSolveArgs a{};
        a.variant = o.variant;
        int bpc = 0;
        int32_t *qv = reinterpret_cast<int32_t *>(base + pl->o_queue);
        VrkQueue qa{};
        if (pl->persistent) qa = VrkQueue{qv, qv + VRK_NQUEUE, qv + 2 * VRK_NQUEUE};
        e = vrk_launch_mfma_solve(a, nullptr, qa, 1, pl->waves, pl->ep, pl->lds, s, 1, &bpc);
        if (e != hipSuccess) return hip_fail(e, "MFMA kernel attributes");
        int bpc_adj = bpc;
        if (pl->adjoint_ready) {
            a.adjoint = 1;
            e = vrk_launch_mfma_solve(a, nullptr, qa, 1, pl->waves_adj, pl->ep_adj, pl->lds_adj, s, 1, &bpc_adj);
            if (e != hipSuccess) return hip_fail(e, "MFMA kernel attributes (adjoint)");
        }
        if (pl->wave_T) {
            int bw = 0;
            e = vrk_launch_wave_solve(a, nullptr, 1, pl->wave_T, pl->wave_bpw, pl->lds_wave, s, 1, &bw);
            if (e != hipSuccess) return hip_fail(e, "wave-owned kernel attributes");
            bpc = bpc_adj = bw;
        }
        int dev = 0, cus = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "device query");
        const int64_t nw = (int64_t)pl->work.size();
        const int64_t g = (int64_t)std::max(1, cus) * std::max(1, bpc);
        const int64_t ga = (int64_t)std::max(1, cus) * std::max(1, bpc_adj);
        pl->grid = pl->persistent ? (int32_t)std::min<int64_t>(g, nw) : (int32_t)nw;
        pl->grid_adj = pl->persistent ? (int32_t)std::min<int64_t>(ga, nw) : (int32_t)nw;
    } else {
        e = pl->small ? vrk_prepare_small_solve(o.dtype, pl->max_nt, pl->lds) : vrk_prepare_vec_solve(o.dtype, pl->lds);
        if (e != hipSuccess) return hip_fail(e, "vector kernel attributes");
    }
    pl->d_ws = base;
    pl->bound = true;
    return VRK_OK;
}

// Workspace owned by the library for callers that cannot allocate device
// memory (vrk_plan_bind_static): one copy on every device the library runs
// on, kept until the process ends. Host code never passes `scratch` itself
// to the device (its name is a host-side stand-in there): it takes the
// device address from hipGetSymbolAddress, once per device, and keeps it.
static __device__ __align__(256) uint8_t scratch[VRK_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct ScratchSlot {
    void *ptr = nullptr;   // device address of `scratch` on this device
    uint64_t gen = 0;      // number of the latest binding to it
};

std::mutex g_scratch_mu;
ScratchSlot g_scratch[kMaxDevices];

// The plan's workspace is still its own: for a scratch binding, no other
// plan has been bound to that device's scratch since.
vrk_status check_bound(const vrk_plan *pl, const char *what)
{
    if (!pl->bound) return fail(VRK_ESTATE, "vrk_plan_bind or vrk_plan_bind_static must precede %s", what);
    if (pl->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch[pl->static_dev].gen != pl->static_gen)
            return fail(VRK_ESTATE,
                        "%s: another plan was bound to the scratch workspace of device %d since this one; "
                        "bind this plan again", what, pl->static_dev);
    }
    return VRK_OK;
}

}  // namespace

extern "C" {

vrk_status vrk_plan_bind(vrk_plan *pl, void *d_ws, size_t ws_bytes, void *stream)
{
    g_err.clear();
    if (!pl) return fail(VRK_EINVAL, "plan null");
    if (!d_ws || ws_bytes < pl->ws_bytes || (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return fail(VRK_EWORKSPACE, "workspace must be >= %zu bytes and 256-byte aligned (got %zu at %p)",
                    pl->ws_bytes, ws_bytes, d_ws);
    pl->static_dev = -1;
    return bind_at(pl, d_ws, stream);
}

vrk_status vrk_plan_bind_static(vrk_plan *pl, void *stream)
{
    g_err.clear();
    if (!pl) return fail(VRK_EINVAL, "plan null");
    if (pl->ws_bytes > VRK_SCRATCH_BYTES)
        return fail(VRK_EWORKSPACE,
                    "the plan needs %zu bytes of workspace, more than the %zu-byte scratch array of "
                    "vrk_plan_bind_static; bind a caller workspace with vrk_plan_bind instead",
                    pl->ws_bytes, (size_t)VRK_SCRATCH_BYTES);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(VRK_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    void *ptr = nullptr;
    uint64_t gen = 0;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ScratchSlot &sl = g_scratch[dev];
        if (!sl.ptr) {
            // first binding on this device (the current one): its copy's address
            e = hipGetSymbolAddress(&sl.ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !sl.ptr) {
                sl.ptr = nullptr;
                return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            }
        }
        ptr = sl.ptr;
        gen = ++sl.gen;   // plans bound to this scratch before are now stale
    }
    pl->static_dev = -1;
    vrk_status st = bind_at(pl, ptr, stream);
    if (st != VRK_OK) return st;
    pl->static_dev = dev;
    pl->static_gen = gen;
    return VRK_OK;
}

static vrk_status run_solve(vrk_plan *pl, void *stream, int32_t *d_iters, float *d_relres,
                            int32_t *d_flags, int adjoint)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    VrkSolveArgs a{};
    a.desc = reinterpret_cast<const VrkDesc *>(pl->d_ws + pl->o_desc);
    a.nprob = (int32_t)pl->pp.size();
    a.max_rhs = pl->max_rhs;
    a.dtype = pl->opt.dtype;
    a.variant = pl->opt.variant;
    a.select = pl->opt.select;
    a.schedule = pl->schedule;
    a.adjoint = adjoint;
    a.tol = pl->opt.tol;
    a.max_iters = pl->opt.max_iters;
    a.check_every = pl->opt.check_every > 0 ? pl->opt.check_every : 1;
    a.seed = pl->opt.seed;
    a.iters = d_iters;
    a.relres = d_relres;
    a.flags = d_flags;
    if (pl->total_rhs == 0) return VRK_OK;
    hipError_t e;
    if (pl->engine == VRK_ENGINE_MFMA) {
        int32_t *qv = reinterpret_cast<int32_t *>(pl->d_ws + pl->o_queue);
        VrkQueue q{};
        if (pl->persistent) q = VrkQueue{qv, qv + VRK_NQUEUE, qv + 2 * VRK_NQUEUE};
        const VrkWork *wl = reinterpret_cast<const VrkWork *>(pl->d_ws + pl->o_work);
        if (pl->wave_T)
            e = vrk_launch_wave_solve(a, wl, (int32_t)pl->work.size(), pl->wave_T, pl->wave_bpw, pl->lds_wave, s, 0,
                                      nullptr);
        else
            e = adjoint ? vrk_launch_mfma_solve(a, wl, q, pl->grid_adj, pl->waves_adj, pl->ep_adj, pl->lds_adj, s, 0,
                                                nullptr)
                        : vrk_launch_mfma_solve(a, wl, q, pl->grid, pl->waves, pl->ep, pl->lds, s, 0, nullptr);
    } else {
        e = pl->small ? vrk_launch_small_solve(a, pl->max_nt, pl->lds, s) : vrk_launch_vec_solve(a, pl->lds, s);
    }
    if (e != hipSuccess) return hip_fail(e, "solve kernel");
    return VRK_OK;
}

vrk_status vrk_plan_refresh(vrk_plan *pl, void *stream)
{
    g_err.clear();
    if (!pl) return fail(VRK_EINVAL, "plan null");
    if (vrk_status st = check_bound(pl, "vrk_plan_refresh")) return st;
    return channel_kernels(pl, pl->d_ws, reinterpret_cast<hipStream_t>(stream));
}

vrk_status vrk_solve(vrk_plan *pl, void *stream, int32_t *d_iters, float *d_relres, int32_t *d_flags)
{
    g_err.clear();
    if (!pl) return fail(VRK_EINVAL, "plan null");
    if (vrk_status st = check_bound(pl, "vrk_solve")) return st;
    return run_solve(pl, stream, d_iters, d_relres, d_flags, 0);
}

vrk_status vrk_solve_adjoint(vrk_plan *pl, void *stream, int32_t *d_iters, float *d_relres,
                             int32_t *d_flags)
{
    g_err.clear();
    if (!pl) return fail(VRK_EINVAL, "plan null");
    if (vrk_status st = check_bound(pl, "vrk_solve_adjoint")) return st;
    if (!pl->adjoint_ready) return fail(VRK_ESTATE, "problems were planned without adjoint buffers");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const VrkDesc *dd = reinterpret_cast<const VrkDesc *>(pl->d_ws + pl->o_desc);
    if (pl->total_rhs == 0) return VRK_OK;
    const bool mf = pl->engine == VRK_ENGINE_MFMA;
    // the MFMA solve and the vector engine's small-channel form form b = H g
    // themselves; the general vector form takes it from a kernel
    hipError_t e = mf || pl->small
                       ? hipSuccess
                       : vrk_launch_adjoint_rhs(dd, (int32_t)pl->pp.size(), pl->max_rhs, pl->opt.dtype, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint right-hand side kernel");
    vrk_status st = run_solve(pl, stream, d_iters, d_relres, d_flags, 1);
    if (st != VRK_OK) return st;
    e = mf ? vrk_launch_adjoint_grads_mfma(dd, reinterpret_cast<const int4 *>(pl->d_ws + pl->o_gtiles),
                                           reinterpret_cast<const int32_t *>(pl->d_ws + pl->o_gorder),
                                           (int32_t)pl->gtiles.size(), pl->gsplit,
                                           reinterpret_cast<const int4 *>(pl->d_ws + pl->o_ctiles),
                                           (int32_t)pl->ctiles.size(), pl->csplit,
                                           reinterpret_cast<const int4 *>(pl->d_ws + pl->o_gruns),
                                           (int32_t)pl->gruns.size(),
                                           reinterpret_cast<float2 *>(pl->d_ws + pl->o_gpart), s)
           : vrk_launch_adjoint_grads(dd, (int32_t)pl->pp.size(), pl->max_k, pl->opt.dtype, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint gradient kernel");
    if (pl->any_gaps) {
        e = vrk_launch_zero_gaps(dd, (int32_t)pl->pp.size(), pl->opt.dtype, s);
        if (e != hipSuccess) return hip_fail(e, "gap kernel");
    }
    return VRK_OK;
}

vrk_status vrk_link_metrics(vrk_plan *pl, const vrk_link_out *out, void *stream)
{
    g_err.clear();
    if (!pl || !out) return fail(VRK_EINVAL, "plan or output table null");
    if (vrk_status st = check_bound(pl, "vrk_link_metrics")) return st;
    const int32_t nprob = (int32_t)pl->pp.size();
    std::vector<VrkLinkOut> tab(nprob);
    for (int32_t i = 0; i < nprob; ++i) {
        const vrk_problem &p = pl->pp[i].p;
        if (p.nrhs != p.k)
            return fail(VRK_EINVAL, "problem %d: link metrics need nrhs == k (S = I_K), got nrhs %d, k %d", i,
                        p.nrhs, p.k);
        if (!out[i].E || !out[i].rate || !out[i].beta)
            return fail(VRK_EINVAL, "problem %d: E, rate and beta must be set", i);
        if (out[i].lde < p.k) return fail(VRK_EINVAL, "problem %d: lde %lld < k %d", i, (long long)out[i].lde, p.k);
        if (!(out[i].noise > 0.0) || !std::isfinite(out[i].noise))
            return fail(VRK_EINVAL, "problem %d: noise (sigma^2 / rho) %g must be finite and > 0", i, out[i].noise);
        tab[i] = VrkLinkOut{out[i].E, out[i].lde, out[i].rate, out[i].beta, out[i].noise};
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    VrkLinkOut *d_out = reinterpret_cast<VrkLinkOut *>(pl->d_ws + pl->o_link);
    // the table goes to the workspace only when it differs from the one there
    // (bind clears the record, since it may bind another workspace)
    hipError_t e = hipSuccess;
    if (pl->link_host.size() != tab.size() ||
        std::memcmp(pl->link_host.data(), tab.data(), sizeof(VrkLinkOut) * nprob) != 0) {
        pl->link_host = tab;
        e = hipMemcpyAsync(d_out, pl->link_host.data(), sizeof(VrkLinkOut) * nprob, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            pl->link_host.clear();
            return hip_fail(e, "hipMemcpyAsync(link output table)");
        }
    }
    e = vrk_launch_link(reinterpret_cast<const VrkDesc *>(pl->d_ws + pl->o_desc), d_out, nprob, pl->max_k,
                        pl->opt.dtype == VRK_C128 ? 1 : 0, pl->engine == VRK_ENGINE_MFMA ? 1 : 0,
                        reinterpret_cast<double *>(pl->d_ws + pl->o_linkpart), s);
    if (e != hipSuccess) return hip_fail(e, "link metric kernels");
    return VRK_OK;
}

int64_t vrk_plan_query(const vrk_plan *pl, int32_t prob, int32_t what, int32_t *out, int64_t cap)
{
    if (!pl || prob < 0 || prob >= (int32_t)pl->pp.size() || cap < 0 || (cap > 0 && !out)) return -1;
    const ProbPlan &q = pl->pp[prob];
    std::vector<int32_t> v;
    switch (what) {
    case VRK_Q_PERM: v = q.perm; break;
    case VRK_Q_FSET: v = q.flist; break;
    case VRK_Q_COLOUR: v = q.colour; break;
    case VRK_Q_XOFF: v = q.xoff; break;
    case VRK_Q_XIDX: v = q.xidx; break;
    case VRK_Q_ENGINE:
        v = {pl->engine, pl->schedule, pl->waves, (int32_t)pl->lds, pl->persistent, pl->grid, pl->ep, pl->gsplit,
             pl->csplit, pl->engine == VRK_ENGINE_MFMA ? pl->waves_adj : pl->waves, pl->wave_T, pl->wave_bpw};
        break;
    case VRK_Q_TILES: v = {(int32_t)q.n_ha, (int32_t)q.n_hg, (int32_t)q.band, (int32_t)q.n_gm}; break;
    case VRK_Q_GRAD: {
        int32_t rmax = 0;
        for (const int4 &r : pl->gruns) rmax = std::max(rmax, r.y);
        v = {(int32_t)pl->gtiles.size(), pl->gsplit, (int32_t)pl->ctiles.size() / std::max(1, pl->csplit),
             pl->csplit, (int32_t)pl->gruns.size(), rmax};
        break;
    }
    default: return -1;
    }
    int64_t n = (int64_t)v.size();
    for (int64_t i = 0; i < std::min(n, cap); ++i) out[i] = v[i];
    return n;
}

void vrk_plan_destroy(vrk_plan *pl) { delete pl; }

const char *vrk_status_string(vrk_status s)
{
    switch (s) {
    case VRK_OK: return "ok";
    case VRK_EINVAL: return "invalid argument";
    case VRK_EUNSUPPORTED: return "unsupported";
    case VRK_EWORKSPACE: return "workspace too small or misaligned";
    case VRK_EHIP: return "HIP runtime error";
    case VRK_ESTATE: return "call order";
    }
    return "unknown status";
}

const char *vrk_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

uint64_t fnv1a(uint64_t hsh, const void *data, size_t n)
{
    const uint8_t *p = static_cast<const uint8_t *>(data);
    for (size_t i = 0; i < n; ++i) {
        hsh ^= p[i];
        hsh *= 1099511628211ULL;
    }
    return hsh;
}

uint64_t shape_key(const vrk_problem *probs, int32_t nprob, const vrk_options &o)
{
    uint64_t hsh = 1469598103934665603ULL;
    int32_t head[4] = {o.variant, o.select, o.dtype, nprob};
    hsh = fnv1a(hsh, head, sizeof head);
    for (int i = 0; i < nprob; ++i) {
        int64_t band = 0;
        for (int k = 0; k < probs[i].k; ++k) band += probs[i].vr_len[k];
        int64_t v[4] = {probs[i].nt, probs[i].k, probs[i].nrhs, band};
        hsh = fnv1a(hsh, v, sizeof v);
        if (probs[i].vr_mask) hsh = fnv1a(hsh, probs[i].vr_mask, sizeof(uint64_t) * probs[i].k);
    }
    return hsh;
}

struct Cand {
    int32_t engine, waves, persistent, schedule;
};

bool cache_lookup(const char *path, uint64_t key, Cand *c, float *ms)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool hit = false;
    while (fgets(line, sizeof line, f)) {
        unsigned long long k;
        Cand t;
        float m;
        if (sscanf(line, "%llx %d %d %d %d %f", &k, &t.engine, &t.waves, &t.persistent, &t.schedule, &m) == 6 &&
            (uint64_t)k == key) {
            *c = t;
            *ms = m;
            hit = true;
        }
    }
    fclose(f);
    return hit;
}

void cache_store(const char *path, uint64_t key, const Cand &c, float ms)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%016llx %d %d %d %d %.6f\n", (unsigned long long)key, c.engine, c.waves, c.persistent,
            c.schedule, ms);
    fclose(f);
}

void apply(vrk_options &o, const Cand &c)
{
    o.engine = c.engine;
    o.tile_waves = c.waves;
    o.persistent = c.persistent;
    o.schedule = c.schedule;
}

}  // namespace

extern "C" vrk_status vrk_autotune(const vrk_problem *probs, int32_t nprob, vrk_options *opt, void *d_ws,
                                   size_t ws_bytes, void *stream, const char *cache_path, int32_t reps,
                                   size_t *ws_needed, float *best_ms)
{
    g_err.clear();
    if (!opt || !probs || nprob < 1) return fail(VRK_EINVAL, "autotune: null options or no problems");
    std::vector<Cand> cands;
    if (opt->dtype == VRK_C64) {
        for (int w : {8, 16})
            for (int per : {0, 1}) cands.push_back({VRK_ENGINE_MFMA, w, per, VRK_SCHED_GATHER});
    }
    cands.push_back({VRK_ENGINE_VECTOR, 0, 0, VRK_SCHED_GATHER});
    cands.push_back({VRK_ENGINE_VECTOR, 0, 0, VRK_SCHED_COLOUR});
    // workspace each candidate needs (host-only planning)
    std::vector<size_t> need(cands.size(), 0);
    std::vector<bool> ok(cands.size(), false);
    size_t maxneed = 0;
    for (size_t c = 0; c < cands.size(); ++c) {
        vrk_options o = *opt;
        apply(o, cands[c]);
        vrk_plan *pl = nullptr;
        size_t ws = 0;
        if (vrk_plan_create(probs, nprob, &o, &ws, &pl) == VRK_OK) {
            ok[c] = true;
            need[c] = ws;
            maxneed = std::max(maxneed, ws);
            vrk_plan_destroy(pl);
        }
    }
    g_err.clear();
    if (ws_needed) *ws_needed = maxneed;
    if (!d_ws) return VRK_OK;
    const uint64_t key = shape_key(probs, nprob, *opt);
    Cand hitc;
    float hitms;
    if (cache_lookup(cache_path, key, &hitc, &hitms)) {
        apply(*opt, hitc);
        if (best_ms) *best_ms = hitms;
        return VRK_OK;
    }
    if (reps < 1) reps = 1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(VRK_EHIP, "autotune: hipEventCreate failed");
    float best = -1.f;
    Cand bestc{};
    vrk_status st = VRK_OK;
    for (size_t c = 0; c < cands.size() && st == VRK_OK; ++c) {
        if (!ok[c] || need[c] > ws_bytes) continue;
        vrk_options o = *opt;
        apply(o, cands[c]);
        vrk_plan *pl = nullptr;
        size_t ws = 0;
        if (vrk_plan_create(probs, nprob, &o, &ws, &pl) != VRK_OK) continue;
        st = vrk_plan_bind(pl, d_ws, ws_bytes, stream);
        if (st == VRK_OK) st = vrk_solve(pl, stream, nullptr, nullptr, nullptr);   // warm-up
        if (st == VRK_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(VRK_EHIP, "autotune: event record");
        for (int r = 0; r < reps && st == VRK_OK; ++r) st = vrk_solve(pl, stream, nullptr, nullptr, nullptr);
        float ms = 0.f;
        if (st == VRK_OK) {
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = fail(VRK_EHIP, "autotune: event timing");
        }
        vrk_plan_destroy(pl);
        if (st != VRK_OK) break;
        ms /= reps;
        if (best < 0.f || ms < best) {
            best = ms;
            bestc = cands[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VRK_OK) return st;
    if (best < 0.f) return fail(VRK_EWORKSPACE, "autotune: no candidate fits the %zu-byte workspace", ws_bytes);
    apply(*opt, bestc);
    if (best_ms) *best_ms = best;
    cache_store(cache_path, key, bestc, best);
    return VRK_OK;
}
