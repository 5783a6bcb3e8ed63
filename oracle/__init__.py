"""FP64 CPU oracle for VR-banded Kaczmarz RZF precoding.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package. It
shares no code with the HIP path (the C source is ``vrk_oracle.c``).

Every function takes numpy arrays in the layout of the channel equation of
Sec. II: ``H`` is ``K x Nt`` complex128 (row k = user k), ``vr_start`` /
``vr_len`` the per-user visibility interval, ``S`` is ``B x K`` (one symbol
vector per row), ``xi`` the RZF regulariser.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

VARIANTS = {"grk": 0, "ahk": 1, "vr_ogrk": 2, "vr_oahk": 3}
SELECT = {"baiwu": 0, "residual": 1, "max": 2, "energy": 3, "uniform": 4}
F_CONVERGED, F_NONFINITE, F_MAXITER = 1, 2, 4


class _Problem(C.Structure):
    _fields_ = [("nt", C.c_int32), ("k", C.c_int32), ("xi", C.c_double),
                ("H", C.c_void_p), ("ldh", C.c_int64),
                ("vs", C.c_void_p), ("vl", C.c_void_p),
                ("mask", C.c_void_p), ("n_sub", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        src = os.path.join(os.path.dirname(LIB), "vrk_oracle.c")
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(src):
            build()
        _lib = C.CDLL(LIB)
        P = C.POINTER(_Problem)
        vp, i32, i64, f64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
        sig = {
            "orc_philox4x64_10": (None, [vp, vp, vp]),
            "orc_uniform24": (f64, [u64, i64, i64, i64]),
            "orc_overlap_sets": (C.c_int, [P, vp, vp]),
            "orc_mis": (C.c_int, [P, vp]),
            "orc_rzf_cholesky": (C.c_int, [P, i32, vp, i64, vp, i64, vp, i64]),
            "orc_rzf_grad": (C.c_int, [P, i32, vp, i64, vp, i64, vp, i64, vp, i64, vp]),
            "orc_kaczmarz": (C.c_int, [P, C.c_int, C.c_int, f64, i64, u64, i64, i64, vp,
                                       vp, vp, vp, vp, vp, vp, vp, i64, vp]),
            "orc_kaczmarz_batch": (C.c_int, [P, C.c_int, C.c_int, f64, i64, u64, i64, i32, vp, i64,
                                             vp, i64, vp, i64, vp, vp, vp]),
            "orc_residual_rows": (None, [P, vp, vp, vp, vp]),
            "orc_row_norms": (None, [P, vp]),
            "orc_step_row": (None, [P, C.c_int, vp, vp, vp]),
            "orc_step_orthogonal": (None, [P, vp, vp, vp, vp]),
            "orc_step_aggregate": (C.c_int, [P, vp, vp, vp, vp]),
            "orc_select": (C.c_int, [C.c_int, C.c_int, vp, vp, f64, f64]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Problem:
    """Keeps the arrays of one drop alive and exposes the C struct."""

    def __init__(self, H, vr_start, vr_len, xi, masks=None, n_sub=0):
        self.H = np.ascontiguousarray(H, dtype=np.complex128)
        self.vs = np.ascontiguousarray(vr_start, dtype=np.int32)
        self.vl = np.ascontiguousarray(vr_len, dtype=np.int32)
        self.k, self.nt = self.H.shape
        self.xi = float(xi)
        self.mask = None if masks is None else np.ascontiguousarray(masks, dtype=np.uint64)
        self.c = _Problem(self.nt, self.k, self.xi, _ptr(self.H), self.nt,
                          _ptr(self.vs), _ptr(self.vl),
                          None if self.mask is None else _ptr(self.mask), int(n_sub))

    @property
    def ref(self):
        return C.byref(self.c)


def _check(st):
    if st != 0:
        raise ValueError("oracle rejected the arguments (status %d)" % st)


def num_threads() -> int:
    """OpenMP threads the batched oracle calls use."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the batched oracle calls from now on (for timing)."""
    _load().orc_set_num_threads(int(n))


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform24(seed: int, step: int, rhs: int, drop: int) -> float:
    return _load().orc_uniform24(seed, step, rhs, drop)


def overlap_sets(H, vr_start, vr_len, xi=1.0, masks=None, n_sub=0):
    """Non-orthogonal sets X_k (including k) as a list of index arrays."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    xoff = np.zeros(p.k + 1, dtype=np.int32)
    xidx = np.zeros(p.k * p.k, dtype=np.int32)
    _check(_load().orc_overlap_sets(p.ref, _ptr(xoff), _ptr(xidx)))
    return [xidx[xoff[i]:xoff[i + 1]].copy() for i in range(p.k)]


def mis(H, vr_start, vr_len, xi=1.0, masks=None, n_sub=0) -> np.ndarray:
    """Boolean mask of the orthogonal set F (maximum independent set)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    m = np.zeros(p.k, dtype=np.uint8)
    _check(_load().orc_mis(p.ref, _ptr(m)))
    return m.astype(bool)


def rzf(H, vr_start, vr_len, S, xi, masks=None, n_sub=0):
    """Closed-form RZF via Cholesky: returns (X, V), X = B x Nt, V = B x K."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    S = np.ascontiguousarray(np.atleast_2d(S), dtype=np.complex128)
    B = S.shape[0]
    X = np.zeros((B, p.nt), dtype=np.complex128)
    V = np.zeros((B, p.k), dtype=np.complex128)
    _check(_load().orc_rzf_cholesky(p.ref, B, _ptr(S), p.k, _ptr(X), p.nt, _ptr(V), p.k))
    return X, V


def rzf_grad(H, vr_start, vr_len, S, xi, G, masks=None, n_sub=0):
    """Closed-form gradient (torch convention) of a real loss whose gradient
    on X is G: returns (gH, gS, gxi)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    S = np.ascontiguousarray(np.atleast_2d(S), dtype=np.complex128)
    G = np.ascontiguousarray(np.atleast_2d(G), dtype=np.complex128)
    B = S.shape[0]
    gH = np.zeros((p.k, p.nt), dtype=np.complex128)
    gS = np.zeros((B, p.k), dtype=np.complex128)
    gxi = np.zeros(1, dtype=np.float64)
    _check(_load().orc_rzf_grad(p.ref, B, _ptr(S), p.k, _ptr(G), p.nt, _ptr(gH), p.nt,
                                _ptr(gS), p.k, _ptr(gxi)))
    return gH, gS, float(gxi[0])


def solve(H, vr_start, vr_len, s, xi, variant="vr_oahk", select="baiwu", tol=1e-10,
          max_iters=100000, seed=0, drop=0, rhs=0, trace=False, masks=None, n_sub=0):
    """One right-hand side. Returns a dict with x, q, iters, relres, flags
    and, with ``trace=True``, z (every iterate [x; q]) and idx (rows chosen,
    -1 / -2 for the F / V half-steps, -3 for z0)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    s = np.ascontiguousarray(s, dtype=np.complex128).reshape(p.k)
    x = np.zeros(p.nt, dtype=np.complex128)
    q = np.zeros(p.k, dtype=np.complex128)
    it = np.zeros(1, dtype=np.int64)
    rel = np.zeros(1, dtype=np.float64)
    fl = np.zeros(1, dtype=np.int32)
    tn = np.zeros(1, dtype=np.int64)
    cap = 2 * max_iters + 1 if trace else 0
    tz = np.zeros((cap, p.nt + p.k), dtype=np.complex128) if trace else None
    ti = np.zeros(cap, dtype=np.int32) if trace else None
    _check(_load().orc_kaczmarz(p.ref, VARIANTS[variant], SELECT[select], tol, max_iters, seed,
                                drop, rhs, _ptr(s), _ptr(x), _ptr(q), _ptr(it), _ptr(rel),
                                _ptr(fl), _ptr(tz) if trace else None,
                                _ptr(ti) if trace else None, cap, _ptr(tn)))
    out = dict(x=x, q=q, iters=int(it[0]), relres=float(rel[0]), flags=int(fl[0]))
    if trace:
        n = int(min(tn[0], cap))
        out["z"] = tz[:n]
        out["idx"] = ti[:n]
    return out


def solve_batch(H, vr_start, vr_len, S, xi, variant="vr_oahk", select="baiwu", tol=1e-5,
                max_iters=100000, seed=0, drop=0, masks=None, n_sub=0):
    """All right-hand sides of one drop (OpenMP over rows of S)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    S = np.ascontiguousarray(np.atleast_2d(S), dtype=np.complex128)
    B = S.shape[0]
    X = np.zeros((B, p.nt), dtype=np.complex128)
    V = np.zeros((B, p.k), dtype=np.complex128)
    it = np.zeros(B, dtype=np.int64)
    rel = np.zeros(B, dtype=np.float64)
    fl = np.zeros(B, dtype=np.int32)
    _check(_load().orc_kaczmarz_batch(p.ref, VARIANTS[variant], SELECT[select], tol, max_iters,
                                      seed, drop, B, _ptr(S), p.k, _ptr(X), p.nt, _ptr(V), p.k,
                                      _ptr(it), _ptr(rel), _ptr(fl)))
    return dict(X=X, V=V, iters=it, relres=rel, flags=fl)


def residual(H, vr_start, vr_len, xi, s, x, q, masks=None, n_sub=0) -> np.ndarray:
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    s = np.ascontiguousarray(s, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    q = np.ascontiguousarray(q, dtype=np.complex128)
    r = np.zeros(p.k, dtype=np.complex128)
    _load().orc_residual_rows(p.ref, _ptr(s), _ptr(x), _ptr(q), _ptr(r))
    return r


def row_norms(H, vr_start, vr_len, xi, masks=None, n_sub=0) -> np.ndarray:
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    nrm = np.zeros(p.k, dtype=np.float64)
    _load().orc_row_norms(p.ref, _ptr(nrm))
    return nrm


def step_row(H, vr_start, vr_len, xi, i, s, x, q, masks=None, n_sub=0):
    """One projection (update) onto row i; returns new (x, q)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    s = np.ascontiguousarray(s, dtype=np.complex128)
    x = np.array(x, dtype=np.complex128)
    q = np.array(q, dtype=np.complex128)
    _load().orc_step_row(p.ref, int(i), _ptr(s), _ptr(x), _ptr(q))
    return x, q


def step_orthogonal(H, vr_start, vr_len, xi, in_f, s, x, q, masks=None, n_sub=0):
    """Proposition 1 step (gamma = 1) over the mask in_f; returns (x, q)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    m = np.ascontiguousarray(in_f, dtype=np.uint8)
    s = np.ascontiguousarray(s, dtype=np.complex128)
    x = np.array(x, dtype=np.complex128)
    q = np.array(q, dtype=np.complex128)
    _load().orc_step_orthogonal(p.ref, _ptr(m), _ptr(s), _ptr(x), _ptr(q))
    return x, q


def step_aggregate(H, vr_start, vr_len, xi, in_set, s, x, q, masks=None, n_sub=0):
    """Aggregated projection (update4) over the mask in_set; returns (x, q)."""
    p = Problem(H, vr_start, vr_len, xi, masks, n_sub)
    m = np.ascontiguousarray(in_set, dtype=np.uint8)
    s = np.ascontiguousarray(s, dtype=np.complex128)
    x = np.array(x, dtype=np.complex128)
    q = np.array(q, dtype=np.complex128)
    _load().orc_step_aggregate(p.ref, _ptr(m), _ptr(s), _ptr(x), _ptr(q))
    return x, q


def select(r, nrm, rule, u) -> int:
    r = np.ascontiguousarray(r, dtype=np.complex128)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    return int(_load().orc_select(len(r), SELECT[rule], _ptr(r), _ptr(nrm), float(nrm.sum()),
                                  float(u)))


# ---------------------------------------------------------------------------
# Precoding matrix and link metrics (signal model and spectral efficiency of
# Sec. II, the RZF precoder and its power budget, Remark 1 for F = H^H V, and
# the NMSE of the simulation section). Plain numpy in FP64.
# ---------------------------------------------------------------------------

def band_channel(H, vr_start, vr_len):
    """H with every entry outside the users' VRs set to zero (the channel the
    solver works on: only VR entries are nonzero)."""
    H = np.asarray(H, dtype=np.complex128)
    K, Nt = H.shape
    n = np.arange(Nt)[None, :]
    vs = np.asarray(vr_start)[:, None]
    ve = vs + np.asarray(vr_len)[:, None]
    return np.where((n >= vs) & (n < ve), H, 0)


def precoder(H, vr_start, vr_len, xi):
    """Unnormalised RZF precoding matrix, transposed: row b is f_b, the
    precoder of user b, i.e. the solution x for s = e_b (Remark 1); K x Nt."""
    K = np.asarray(H).shape[0]
    X, _ = rzf(H, vr_start, vr_len, np.eye(K, dtype=np.complex128), xi)
    return X


def link_metrics(H, vr_start, vr_len, noise, X):
    """Link metrics of the precoder whose transposed columns are the rows of
    X (K x Nt). Returns (E, beta, rate):
      E[u, b] = h_u^H f_b = sum over n in VR_u of H[u, n] X[b, n],
      beta    = 1 / ||F||_F  (the power budget ||beta F||_F^2 <= 1 met with
                equality),
      rate[u] = log2(1 + rho beta^2 |E_uu|^2 / (rho beta^2 sum_{b != u}
                |E_ub|^2 + sigma^2)), written with noise = sigma^2 / rho."""
    X = np.asarray(X, dtype=np.complex128)
    E = band_channel(H, vr_start, vr_len) @ X.T
    beta = 1.0 / np.linalg.norm(X)
    a2 = np.abs(E) ** 2
    sig = np.diag(a2).copy()
    intf = a2.sum(axis=1) - sig
    rate = np.log2(1.0 + beta ** 2 * sig / (beta ** 2 * intf + noise))
    return E, beta, rate


def nmse(F_ref, F):
    """||F_ref - F||_F / ||F_ref||_F, the NMSE of the simulation section."""
    F_ref = np.asarray(F_ref)
    return float(np.linalg.norm(F_ref - np.asarray(F)) / np.linalg.norm(F_ref))


# ---------------------------------------------------------------------------
# Subarray VR model of Sec. II: the array is split into S subarrays of
# Nt / S antennas and user k sees the subarrays of M_k, so its VR is their
# union. Masks are per-user integers, bit s set when subarray s is visible;
# every function above takes them as ``masks`` (with ``n_sub`` = S), the
# VR interval then being the hull of the visible subarrays. The two
# definitions below are plain numpy, for the tests.
# ---------------------------------------------------------------------------

def mask_indicator(masks, nt, n_sub):
    """K x Nt 0/1 matrix of the VR indicator vectors u_k (eq. VR)."""
    L = nt // n_sub
    U = np.zeros((len(masks), nt), dtype=np.int8)
    for k, m in enumerate(masks):
        for s in range(n_sub):
            if (int(m) >> s) & 1:
                U[k, s * L:(s + 1) * L] = 1
    return U


def mask_graph(masks):
    """Adjacency of the VR graph: an edge between users that share a visible
    subarray (|M_i cap M_j| > 0), no self loops."""
    K = len(masks)
    A = np.zeros((K, K), dtype=bool)
    for i in range(K):
        for j in range(K):
            A[i, j] = i != j and (int(masks[i]) & int(masks[j])) != 0
    return A

