"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numpy /
scipy library routines, brute force on tiny inputs, exact rational
arithmetic, closed forms of special cases, and the exact invariants the
paper proves (Lemma 2, Theorem 2, Theorem 4, Proposition 1, Lemma 3).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from tests.helpers import augmented, qpsk, random_problem, rzf_numpy


# --------------------------------------------------------------------------
# Philox4x64-10: pinned to numpy.random.Philox (same generator, 10 rounds).
# numpy increments its 256-bit counter before producing a block, so its
# first block for counter c is Philox(c + 1).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((7, 0), (5, 6, 7, 0)),
    ((2**64 - 1, 12345), (2**64 - 1, 3, 9, 1)),
    ((0xDEADBEEF, 0), (1000, 17, 3, 0)),
])
def test_philox_matches_numpy(key, ctr):
    c = np.array(ctr, dtype=np.uint64)
    # numpy's counter carries across words; build c - 1 with borrow
    words = [int(v) for v in ctr]
    val = sum(w << (64 * i) for i, w in enumerate(words))
    prev = (val - 1) % (1 << 256)
    prev_words = np.array([(prev >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev_words)
    want = g.random_raw(4)
    got = oracle.philox4x64_10(c, np.array(key, dtype=np.uint64))
    assert [int(a) for a in got] == [int(b) for b in want]


def test_uniform24_is_top_bits_of_philox():
    for step, rhs, drop in [(0, 0, 0), (5, 3, 2), (123456, 4095, 511)]:
        out = oracle.philox4x64_10(np.array([step, rhs, drop, 0], dtype=np.uint64),
                                   np.array([99, 0], dtype=np.uint64))
        u = oracle.uniform24(99, step, rhs, drop)
        assert u == (int(out[0]) >> 40) / 2.0**24
        assert 0.0 <= u < 1.0


# --------------------------------------------------------------------------
# Closed-form RZF (precoding equation; Theorem 1; Remark 1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("nt,k,seed", [(64, 8, 0), (128, 16, 1), (40, 48, 2), (256, 1, 3), (96, 12, 4)])
def test_rzf_cholesky_matches_numpy_and_scipy(nt, k, seed):
    rng = np.random.default_rng(seed)
    H, vs, vl, xi = random_problem(rng, nt, k)
    S = qpsk(rng, (5, k))
    X, V = oracle.rzf(H, vs, vl, S, xi)
    Xn, Vn = rzf_numpy(H, S, xi)
    np.testing.assert_allclose(X, Xn, rtol=0, atol=1e-12 * np.abs(Xn).max())
    np.testing.assert_allclose(V, Vn, rtol=0, atol=1e-12 * np.abs(Vn).max())
    M = H @ H.conj().T + xi * np.eye(k)
    c = scipy.linalg.cho_factor(M, lower=True)
    Vs = scipy.linalg.cho_solve(c, S.T).T
    np.testing.assert_allclose(V, Vs, rtol=0, atol=1e-12 * np.abs(Vs).max())


def test_min_norm_bruteforce_tiny():
    """Theorem 1 + Remark 1: the min-norm solution of [H, sqrt(xi) I] z = s
    (pinv, brute force) has x in its first Nt entries and sqrt(xi) v in the
    last K."""
    rng = np.random.default_rng(10)
    for nt, k in [(16, 4), (24, 8), (8, 8), (6, 10)]:
        H, vs, vl, xi = random_problem(rng, nt, k, lo=2, hi=nt)
        s = qpsk(rng, (k,))
        z = np.linalg.pinv(augmented(H, xi)) @ s
        X, V = oracle.rzf(H, vs, vl, s, xi)
        np.testing.assert_allclose(X[0], z[:nt], atol=1e-12)
        np.testing.assert_allclose(V[0], z[nt:] / np.sqrt(xi), atol=1e-12)


def test_least_squares_form_appendix_a():
    """Appendix A: v = argmin ||G v - g||, G = [H^H; sqrt(xi) I] (paper
    orientation), g = [0; s / sqrt(xi)]."""
    rng = np.random.default_rng(11)
    H, vs, vl, xi = random_problem(rng, 48, 6)
    s = qpsk(rng, (6,))
    G = np.vstack([H.conj().T, np.sqrt(xi) * np.eye(6)])
    g = np.concatenate([np.zeros(48), s / np.sqrt(xi)])
    v = np.linalg.lstsq(G, g, rcond=None)[0]
    _, V = oracle.rzf(H, vs, vl, s, xi)
    np.testing.assert_allclose(V[0], v, atol=1e-12)


def _gauss_solve_exact(M, b):
    """Gauss-Jordan over Gaussian rationals (pairs of Fractions)."""
    n = len(b)
    A = [[M[i][j] for j in range(n)] + [b[i]] for i in range(n)]

    def mul(a, c):
        return (a[0] * c[0] - a[1] * c[1], a[0] * c[1] + a[1] * c[0])

    def inv(a):
        d = a[0] * a[0] + a[1] * a[1]
        return (a[0] / d, -a[1] / d)

    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != (0, 0))
        A[c], A[piv] = A[piv], A[c]
        iv = inv(A[c][c])
        A[c] = [mul(iv, e) for e in A[c]]
        for r in range(n):
            if r != c and A[r][c] != (0, 0):
                f = A[r][c]
                A[r] = [(A[r][j][0] - mul(f, A[c][j])[0], A[r][j][1] - mul(f, A[c][j])[1])
                        for j in range(n + 1)]
    return [A[i][n] for i in range(n)]


def test_rzf_exact_rational_small_integer_channel():
    """Integer channel entries, xi = 1: v = (H H^H + I)^-1 s and x = H^H v
    computed exactly in rational arithmetic."""
    Hi = [[(1, 2), (0, -1), (3, 0), (0, 0), (0, 0)],
          [(0, 0), (2, 1), (-1, 1), (1, 0), (0, 0)],
          [(0, 0), (0, 0), (0, 0), (1, -2), (2, 2)]]
    vs = np.array([0, 1, 3], dtype=np.int32)
    vl = np.array([3, 3, 2], dtype=np.int32)
    s = [(1, 1), (-1, 1), (1, -1)]
    K, N = 3, 5
    Fr = [[(Fraction(a), Fraction(b)) for (a, b) in row] for row in Hi]
    M = []
    for i in range(K):
        row = []
        for j in range(K):
            re = sum(Fr[i][n][0] * Fr[j][n][0] + Fr[i][n][1] * Fr[j][n][1] for n in range(N))
            im = sum(Fr[i][n][1] * Fr[j][n][0] - Fr[i][n][0] * Fr[j][n][1] for n in range(N))
            row.append((re + (1 if i == j else 0), im))
        M.append(row)
    v = _gauss_solve_exact(M, [(Fraction(a), Fraction(b)) for a, b in s])
    x = []
    for n in range(N):
        re = sum(Fr[k][n][0] * v[k][0] + Fr[k][n][1] * v[k][1] for k in range(K))
        im = sum(Fr[k][n][0] * v[k][1] - Fr[k][n][1] * v[k][0] for k in range(K))
        x.append(complex(float(re), float(im)))
    H = np.array([[complex(a, b) for a, b in row] for row in Hi])
    X, V = oracle.rzf(H, vs, vl, np.array([complex(a, b) for a, b in s]), 1.0)
    np.testing.assert_allclose(X[0], np.array(x), rtol=0, atol=1e-14)
    np.testing.assert_allclose(V[0], np.array([complex(float(a), float(b)) for a, b in v]), atol=1e-14)


def test_rzf_special_cases():
    rng = np.random.default_rng(12)
    # K = 1: x = conj(h) s / (||h||^2 + xi), one projection is exact
    H, vs, vl, xi = random_problem(rng, 64, 1)
    s = np.array([0.3 - 0.7j])
    X, _ = oracle.rzf(H, vs, vl, s, xi)
    np.testing.assert_allclose(X[0], H[0].conj() * s[0] / (np.vdot(H[0], H[0]).real + xi), atol=1e-15)
    o = oracle.solve(H, vs, vl, s, xi, variant="grk", tol=1e-14)
    assert o["iters"] == 1
    np.testing.assert_allclose(o["x"], X[0], atol=1e-15)
    # disjoint VRs: H H^H diagonal, x = sum_k conj(h_k) s_k / (||h_k||^2 + xi)
    H, vs, vl, xi = random_problem(rng, 128, 8, disjoint=True)
    s = qpsk(rng, (8,))
    X, V = oracle.rzf(H, vs, vl, s, xi)
    want = sum(H[k].conj() * s[k] / (np.vdot(H[k], H[k]).real + xi) for k in range(8))
    np.testing.assert_allclose(X[0], want, atol=1e-14)
    # large xi: x ~ H^H s / xi (MRC limit)
    H, vs, vl, _ = random_problem(rng, 64, 8)
    s = qpsk(rng, (8,))
    X, _ = oracle.rzf(H, vs, vl, s, 1e9)
    np.testing.assert_allclose(X[0] * 1e9, H.conj().T @ s, rtol=1e-6, atol=1e-9)
    # small xi approaches ZF when H has full row rank
    X, _ = oracle.rzf(H, vs, vl, s, 1e-10)
    zf = H.conj().T @ np.linalg.solve(H @ H.conj().T, s)
    np.testing.assert_allclose(X[0], zf, rtol=0, atol=1e-6 * np.abs(zf).max())
    # zero-length VR: that row is [0, sqrt(xi) e_k], so v_k = s_k / xi
    H, vs, vl, xi = random_problem(rng, 64, 6)
    vl[2] = 0
    H[2] = 0
    s = qpsk(rng, (6,))
    _, V = oracle.rzf(H, vs, vl, s, xi)
    assert abs(V[0, 2] - s[2] / xi) < 1e-14


# --------------------------------------------------------------------------
# VR structure: X_k and the orthogonal set F
# --------------------------------------------------------------------------
def test_overlap_sets_match_structural_gram():
    """X_k = users whose channel rows are structurally non-orthogonal to
    row k (Lemma 1), read off the support of H."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        H, vs, vl, xi = random_problem(rng, 50, 9, lo=0, hi=20)
        sup = np.abs(H) > 0
        got = oracle.overlap_sets(H, vs, vl)
        for k in range(9):
            want = {j for j in range(9) if j == k or np.any(sup[k] & sup[j])}
            assert set(got[k].tolist()) == want


def _brute_mis_size(vs, vl):
    k = len(vs)
    best = 0
    for m in range(1, 1 << k):
        idx = [i for i in range(k) if m >> i & 1]
        ok = all(max(vs[a], vs[b]) >= min(vs[a] + vl[a], vs[b] + vl[b])
                 for a, b in itertools.combinations(idx, 2))
        if ok:
            best = max(best, len(idx))
    return best


def test_mis_is_maximum_independent_set_bruteforce():
    """Problem max_set: F is independent and as large as brute force finds."""
    rng = np.random.default_rng(14)
    for trial in range(60):
        k = int(rng.integers(1, 11))
        H, vs, vl, xi = random_problem(rng, 40, k, lo=0, hi=25)
        f = oracle.mis(H, vs, vl)
        idx = np.flatnonzero(f)
        for a, b in itertools.combinations(idx, 2):
            assert max(vs[a], vs[b]) >= min(vs[a] + vl[a], vs[b] + vl[b])
        assert len(idx) == _brute_mis_size(vs, vl)


# --------------------------------------------------------------------------
# Iterations converge to the pinned RZF for every variant, rule and seed
# --------------------------------------------------------------------------
@pytest.mark.parametrize("variant", ["grk", "ahk", "vr_ogrk", "vr_oahk"])
@pytest.mark.parametrize("rule", ["baiwu", "residual", "max", "energy", "uniform"])
def test_iterations_converge_to_rzf(variant, rule):
    rng = np.random.default_rng(15)
    H, vs, vl, xi = random_problem(rng, 96, 12)
    for seed in range(3):
        s = qpsk(rng, (12,))
        X, _ = oracle.rzf(H, vs, vl, s, xi)
        o = oracle.solve(H, vs, vl, s, xi, variant=variant, select=rule, tol=1e-12, seed=seed)
        assert o["flags"] == oracle.F_CONVERGED
        assert np.linalg.norm(o["x"] - X[0]) <= 1e-10 * np.linalg.norm(X[0])


def test_disjoint_vrs_one_iteration_and_k_steps():
    """Theorem 4 / Prop. 1 with F = all users: VR-OAHK converges in one
    iteration; the max rule fixes each row once (Theorem 2), so it needs
    exactly one step per nonzero symbol."""
    rng = np.random.default_rng(16)
    H, vs, vl, xi = random_problem(rng, 160, 10, disjoint=True)
    s = qpsk(rng, (10,))
    s[3] = 0
    X, _ = oracle.rzf(H, vs, vl, s, xi)
    assert oracle.mis(H, vs, vl).all()
    o = oracle.solve(H, vs, vl, s, xi, variant="vr_oahk", tol=1e-13)
    assert o["iters"] == 1 and o["flags"] == oracle.F_CONVERGED
    np.testing.assert_allclose(o["x"], X[0], atol=1e-14)
    o = oracle.solve(H, vs, vl, s, xi, variant="grk", select="max", tol=1e-13)
    assert o["iters"] == 9
    np.testing.assert_allclose(o["x"], X[0], atol=1e-14)


# --------------------------------------------------------------------------
# Exact invariants of the paper
# --------------------------------------------------------------------------
def _zstar(H, vs, vl, s, xi):
    X, V = oracle.rzf(H, vs, vl, s, xi)
    return np.concatenate([X[0], np.sqrt(xi) * V[0]])


def _zz(z, nt, xi):
    """trace rows hold [x; q]; z-space is [x; sqrt(xi) q]."""
    return np.concatenate([z[:nt], np.sqrt(xi) * z[nt:]])


@pytest.mark.parametrize("variant,rule", [("grk", "baiwu"), ("vr_ogrk", "residual"),
                                          ("ahk", "baiwu"), ("vr_oahk", "baiwu"), ("grk", "max")])
def test_pythagorean_identity_every_step(variant, rule):
    """Lemma 2 / (gougu) and Lemma 3 / (gougu2): in z-space,
    ||e_{t+1}||^2 = ||e_t||^2 - ||z_{t+1} - z_t||^2 at every (half-)step."""
    rng = np.random.default_rng(17)
    H, vs, vl, xi = random_problem(rng, 80, 10)
    s = qpsk(rng, (10,))
    zs = _zstar(H, vs, vl, s, xi)
    o = oracle.solve(H, vs, vl, s, xi, variant=variant, select=rule, tol=1e-12, trace=True, seed=3)
    Z = np.array([_zz(z, 80, xi) for z in o["z"]])
    e2 = np.sum(np.abs(Z - zs) ** 2, axis=1)
    d2 = np.sum(np.abs(np.diff(Z, axis=0)) ** 2, axis=1)
    assert len(Z) > 3
    np.testing.assert_allclose(e2[1:], e2[:-1] - d2, rtol=0, atol=1e-12 * e2[0])
    assert np.all(np.diff(e2) <= 1e-14 * e2[0])


def test_theorem2_orthogonal_rows_keep_residual_bitwise():
    """Theorem 2: after projecting row i, rows orthogonal to it keep their
    residual exactly (checked bit for bit in FP64 with numpy)."""
    rng = np.random.default_rng(18)
    H, vs, vl, xi = random_problem(rng, 120, 12, lo=10, hi=40)
    s = qpsk(rng, (12,))
    o = oracle.solve(H, vs, vl, s, xi, variant="grk", tol=1e-12, trace=True, seed=1)
    xsets = oracle.overlap_sets(H, vs, vl)
    nt = 120
    checked = 0
    for t in range(1, len(o["z"])):
        i = o["idx"][t]
        z0, z1 = o["z"][t - 1], o["z"][t]
        r0 = s - H @ z0[:nt] - xi * z0[nt:]
        r1 = s - H @ z1[:nt] - xi * z1[nt:]
        for j in range(12):
            if j not in xsets[i]:
                assert r0[j] == r1[j]
                checked += 1
    assert checked > 50


def test_theorem4_orthogonal_half_step_solves_f_rows():
    """Theorem 4: after the aggregated step over the mutually orthogonal
    set F, A_F z = s_F holds (to rounding)."""
    rng = np.random.default_rng(19)
    H, vs, vl, xi = random_problem(rng, 200, 14, lo=20, hi=60)
    s = qpsk(rng, (14,))
    f = oracle.mis(H, vs, vl)
    assert f.sum() >= 2
    o = oracle.solve(H, vs, vl, s, xi, variant="vr_oahk", tol=1e-12, trace=True)
    nt = 200
    n_half = 0
    for t in range(len(o["z"])):
        if o["idx"][t] == -1:
            z = o["z"][t]
            r = s - H @ z[:nt] - xi * z[nt:]
            assert np.abs(r[f]).max() <= 1e-13
            n_half += 1
    assert n_half >= 2


def test_proposition1_sequential_equals_grouped():
    """Prop. 1 / Appendix D: single-row projections over disjoint rows, one
    after another, equal the grouped step with gamma = 1."""
    rng = np.random.default_rng(20)
    H, vs, vl, xi = random_problem(rng, 150, 12, lo=10, hi=50)
    s = qpsk(rng, (12,))
    f = oracle.mis(H, vs, vl)
    x = (rng.standard_normal(150) + 1j * rng.standard_normal(150)) * 0.1
    q = (rng.standard_normal(12) + 1j * rng.standard_normal(12)) * 0.1
    xg, qg = oracle.step_orthogonal(H, vs, vl, xi, f, s, x, q)
    xs, qs = x.copy(), q.copy()
    for i in np.flatnonzero(f)[::-1]:
        xs, qs = oracle.step_row(H, vs, vl, xi, i, s, xs, qs)
    np.testing.assert_allclose(xg, xs, rtol=0, atol=1e-15)
    np.testing.assert_allclose(qg, qs, rtol=0, atol=1e-15)
    # and the general aggregated step restricted to F gives the same move
    xa, qa = oracle.step_aggregate(H, vs, vl, xi, f, s, x, q)
    np.testing.assert_allclose(xa, xg, rtol=0, atol=1e-14)
    np.testing.assert_allclose(qa, qg, rtol=0, atol=1e-14)


def test_aggregate_with_unit_coefficient_is_single_row_step():
    """(update4) with phi = e_i reduces to the Kaczmarz update (update)."""
    rng = np.random.default_rng(21)
    H, vs, vl, xi = random_problem(rng, 64, 8)
    s = qpsk(rng, (8,))
    x = rng.standard_normal(64) * 0.1 + 0j
    q = rng.standard_normal(8) * 0.1 + 0j
    for i in range(8):
        m = np.zeros(8, dtype=bool)
        m[i] = True
        xa, qa = oracle.step_aggregate(H, vs, vl, xi, m, s, x, q)
        xr, qr = oracle.step_row(H, vs, vl, xi, i, s, x, q)
        np.testing.assert_allclose(xa, xr, rtol=0, atol=1e-15)
        np.testing.assert_allclose(qa, qr, rtol=0, atol=1e-15)


def test_aggregated_step_decrease_and_rate():
    """(update4): the z-space error drops by exactly (phi^H r)^2/||A^H phi||^2
    and the per-step factor is < 1 whenever r != 0 (Theorem 5's alpha)."""
    rng = np.random.default_rng(22)
    H, vs, vl, xi = random_problem(rng, 90, 10)
    s = qpsk(rng, (10,))
    zs = _zstar(H, vs, vl, s, xi)
    A = augmented(H, xi)
    nrm = np.sum(np.abs(A) ** 2, axis=1)
    x = np.zeros(90, complex)
    q = np.zeros(10, complex)
    allm = np.ones(10, dtype=bool)
    for _ in range(6):
        z = np.concatenate([x, np.sqrt(xi) * q])
        r = s - A @ z
        phi = r / nrm
        pred = np.vdot(phi, r).real ** 2 / np.sum(np.abs(A.conj().T @ phi) ** 2)
        x, q = oracle.step_aggregate(H, vs, vl, xi, allm, s, x, q)
        z1 = np.concatenate([x, np.sqrt(xi) * q])
        e0 = np.sum(np.abs(z - zs) ** 2)
        e1 = np.sum(np.abs(z1 - zs) ** 2)
        assert abs((e0 - e1) - pred) <= 1e-12 * e0
        assert e1 < e0


def test_selection_rules_against_definitions():
    """Threshold-and-sample selection: with u swept over [0, 1), the
    BAIWU rule picks exactly the rows with |r_i|^2 >= eps ||r||^2 ||a_i||^2
    (eps as in the cited greedy randomized Kaczmarz), each with probability
    |r_i|^2 / sum_U |r_j|^2; RESIDUAL uses every row with |r_i|^2/||r||^2;
    MAX picks the largest |r_i|^2/||a_i||^2."""
    rng = np.random.default_rng(23)
    for _ in range(10):
        K = 12
        r = (rng.standard_normal(K) + 1j * rng.standard_normal(K)) * rng.random(K) ** 3
        nrm = rng.random(K) + 0.5
        w = np.abs(r) ** 2
        eps = 0.5 * (np.max(w / nrm) / w.sum() + 1.0 / nrm.sum())
        U = set(np.flatnonzero(w >= eps * w.sum() * nrm).tolist())
        us = (np.arange(4096) + 0.5) / 4096
        picks = np.array([oracle.select(r, nrm, "baiwu", u) for u in us])
        assert set(picks.tolist()) == U
        wu = np.array([w[i] if i in U else 0.0 for i in range(K)])
        freq = np.bincount(picks, minlength=K) / len(us)
        np.testing.assert_allclose(freq, wu / wu.sum(), atol=2.0 / 4096)
        picks = np.array([oracle.select(r, nrm, "residual", u) for u in us])
        freq = np.bincount(picks, minlength=K) / len(us)
        np.testing.assert_allclose(freq, w / w.sum(), atol=2.0 / 4096)
        assert oracle.select(r, nrm, "max", 0.3) == int(np.argmax(w / nrm))


def test_randomized_criteria_against_definitions():
    """Sec. III-A's criteria: with u swept over [0, 1), ENERGY picks row i
    with frequency ||a_i||^2 / ||A||_F^2 and UNIFORM with 1/K, whatever the
    residual (a zero residual included)."""
    rng = np.random.default_rng(26)
    us = (np.arange(4096) + 0.5) / 4096
    for _ in range(10):
        K = int(rng.integers(2, 20))
        r = (rng.standard_normal(K) + 1j * rng.standard_normal(K)) * rng.random(K) ** 3
        nrm = rng.random(K) * 3 + 0.1
        for rr in (r, np.zeros(K, dtype=complex)):
            pe = np.array([oracle.select(rr, nrm, "energy", u) for u in us])
            np.testing.assert_allclose(np.bincount(pe, minlength=K) / len(us), nrm / nrm.sum(), atol=2.0 / 4096)
            pu = np.array([oracle.select(rr, nrm, "uniform", u) for u in us])
            np.testing.assert_allclose(np.bincount(pu, minlength=K) / len(us), np.full(K, 1.0 / K), atol=2.0 / 4096)
        # the first row whose inclusive prefix exceeds u times the total
        u = 0.37
        assert oracle.select(r, nrm, "energy", u) == int(np.argmax(np.cumsum(nrm) > u * nrm.sum()))


def test_randomized_criteria_expected_decrease():
    """One single-row step from a common state, averaged over the sampling
    (u swept over [0, 1)): the energy criterion removes on average exactly
    ||r||^2 / ||A||_F^2 of the squared error (Strohmer and Vershynin's
    identity, each row's decrease being |r_i|^2 / ||a_i||^2 by the
    Pythagorean identity), the uniform one (1/K) sum_i |r_i|^2 / ||a_i||^2;
    both at least sigma_min(A)^2 ||e||^2 / (K max_i ||a_i||^2)."""
    rng = np.random.default_rng(27)
    H, vs, vl, xi = random_problem(rng, 60, 9)
    H[:, :] *= np.linspace(0.3, 2.0, 9)[:, None]   # unequal row energies
    s = qpsk(rng, (9,))
    zs = _zstar(H, vs, vl, s, xi)
    o = oracle.solve(H, vs, vl, s, xi, variant="vr_oahk", tol=0.0, max_iters=1)
    x0, q0 = o["x"], o["q"]
    e0 = np.sum(np.abs(_zz(np.concatenate([x0, q0]), 60, xi) - zs) ** 2)
    r = oracle.residual(H, vs, vl, xi, s, x0, q0)
    nrm = oracle.row_norms(H, vs, vl, xi)
    A = augmented(H, xi)
    sig_min = np.linalg.svd(A, compute_uv=False)[-1]
    us = (np.arange(2048) + 0.5) / 2048
    for rule, want in (("energy", np.sum(np.abs(r) ** 2) / nrm.sum()),
                       ("uniform", np.mean(np.abs(r) ** 2 / nrm))):
        dec = []
        for u in us:
            i = oracle.select(r, nrm, rule, u)
            x1, q1 = oracle.step_row(H, vs, vl, xi, i, s, x0, q0)
            dec.append(e0 - np.sum(np.abs(_zz(np.concatenate([x1, q1]), 60, xi) - zs) ** 2))
        # the sweep's frequencies differ from p_i by at most 1/2048 per row
        slack = 2.0 / 2048 * np.sum(np.abs(r) ** 2 / nrm)
        assert abs(np.mean(dec) - want) <= slack, (rule, np.mean(dec), want)
        assert want >= sig_min ** 2 * e0 / (9 * nrm.max()) * (1 - 1e-12)


def test_theorem3_rate_bound():
    """Theorem 3 (as corrected): per step, ||e_{t+1}||^2 <= (1 -
    sigma_min(A)^2/||A||_F^2) ||e_t||^2. For the threshold and max rules it
    holds at every step; for the residual-proportional rule it holds in
    expectation (averaged over seeds from a common state)."""
    rng = np.random.default_rng(24)
    H, vs, vl, xi = random_problem(rng, 70, 10)
    A = augmented(H, xi)
    sig = np.linalg.svd(A, compute_uv=False)
    eta = 1.0 - sig[-1] ** 2 / np.sum(np.abs(A) ** 2)
    s = qpsk(rng, (10,))
    zs = _zstar(H, vs, vl, s, xi)
    for rule in ["baiwu", "max"]:
        for seed in range(5):
            o = oracle.solve(H, vs, vl, s, xi, variant="grk", select=rule, tol=1e-12, trace=True,
                             seed=seed)
            e2 = np.array([np.sum(np.abs(_zz(z, 70, xi) - zs) ** 2) for z in o["z"]])
            assert np.all(e2[1:] <= eta * e2[:-1] * (1 + 1e-9) + 1e-28)
    # expectation for the residual rule: one step from a common state
    o = oracle.solve(H, vs, vl, s, xi, variant="grk", select="residual", tol=0.0, max_iters=5,
                     trace=True)
    z5 = o["z"][-1]
    e0 = np.sum(np.abs(_zz(z5, 70, xi) - zs) ** 2)
    r = s - H @ z5[:70] - xi * z5[70:]
    nrm = oracle.row_norms(H, vs, vl, xi)
    drops = []
    for seed in range(400):
        i = oracle.select(r, nrm, "residual", oracle.uniform24(seed, 0, 0, 0))
        x1, q1 = oracle.step_row(H, vs, vl, xi, i, s, z5[:70], z5[70:])
        drops.append(np.sum(np.abs(_zz(np.concatenate([x1, q1]), 70, xi) - zs) ** 2))
    assert np.mean(drops) <= eta * e0


def test_iteration_count_ordering():
    """Qualitative claim of the simulation section: the aggregated method
    needs far fewer iterations than the single-row greedy method."""
    rng = np.random.default_rng(25)
    H, vs, vl, xi = random_problem(rng, 256, 24, lo=40, hi=120)
    s = qpsk(rng, (24,))
    a = oracle.solve(H, vs, vl, s, xi, variant="vr_ogrk", tol=1e-6)["iters"]
    b = oracle.solve(H, vs, vl, s, xi, variant="vr_oahk", tol=1e-6)["iters"]
    assert b * 3 < a


# --------------------------------------------------------------------------
# Flags and degenerate inputs
# --------------------------------------------------------------------------
def test_flags_and_degenerate_inputs():
    rng = np.random.default_rng(26)
    H, vs, vl, xi = random_problem(rng, 64, 8)
    o = oracle.solve(H, vs, vl, np.zeros(8), xi, variant="grk")
    assert o["iters"] == 0 and o["flags"] == oracle.F_CONVERGED and not o["x"].any()
    s = qpsk(rng, (8,))
    o = oracle.solve(H, vs, vl, s, xi, variant="ahk", tol=1e-12, max_iters=1)
    assert o["iters"] == 1 and o["flags"] == oracle.F_MAXITER
    Hn = H.copy()
    Hn[2, vs[2]] = np.nan
    o = oracle.solve(Hn, vs, vl, s, xi, variant="vr_oahk")
    assert o["flags"] & oracle.F_NONFINITE
    with pytest.raises(ValueError):
        oracle.solve(H, vs, vl, s, 0.0)
    bad = vs.copy()
    bad[0] = 64 - vl[0] + 1
    with pytest.raises(ValueError):
        oracle.solve(H, bad, vl, s, xi)


# --------------------------------------------------------------------------
# Gradient of the closed form: finite differences and torch autograd
# --------------------------------------------------------------------------
def _loss_and_explicit(H, S, X, lam):
    """L = mean_b ||H x_b - s_b||^2 + lam ||x_b||^2 with its torch-convention
    gradient on X (G) and its explicit parts on H and S."""
    B = S.shape[0]
    R = X @ H.T - S                          # rows: H x_b - s_b
    L = (np.sum(np.abs(R) ** 2) + lam * np.sum(np.abs(X) ** 2)) / B
    G = 2.0 * (R @ H.conj() + lam * X) / B   # 2 dL/d conj(x)
    gH_exp = 2.0 * R.T @ X.conj() / B        # 2 dL/d conj(H) holding x fixed
    gS_exp = -2.0 * R / B
    return L, G, gH_exp, gS_exp


def test_rzf_gradient_matches_finite_differences():
    rng = np.random.default_rng(27)
    nt, k, lam = 64, 8, 0.1
    H, vs, vl, xi = random_problem(rng, nt, k)
    S = qpsk(rng, (4, k))

    def total(Hc, Sc, xic):
        X, _ = oracle.rzf(Hc, vs, vl, Sc, xic)
        return _loss_and_explicit(Hc, Sc, X, lam)[0]

    X, _ = oracle.rzf(H, vs, vl, S, xi)
    L, G, gHe, gSe = _loss_and_explicit(H, S, X, lam)
    gH, gS, gxi = oracle.rzf_grad(H, vs, vl, S, xi, G)
    gH = gH + gHe * (np.abs(H) > 0)
    gS = gS + gSe
    h = 1e-6
    for (kk, n) in [(0, vs[0]), (3, vs[3] + vl[3] // 2), (7, vs[7] + vl[7] - 1)]:
        for part, unit in [("re", 1.0), ("im", 1j)]:
            Hp, Hm = H.copy(), H.copy()
            Hp[kk, n] += h * unit
            Hm[kk, n] -= h * unit
            fd = (total(Hp, S, xi) - total(Hm, S, xi)) / (2 * h)
            want = gH[kk, n].real if part == "re" else gH[kk, n].imag
            assert abs(fd - want) <= 1e-7 * max(1.0, abs(want))
    for (b, kk) in [(0, 0), (3, 5)]:
        for unit in [1.0, 1j]:
            Sp, Sm = S.copy(), S.copy()
            Sp[b, kk] += h * unit
            Sm[b, kk] -= h * unit
            fd = (total(H, Sp, xi) - total(H, Sm, xi)) / (2 * h)
            want = gS[b, kk].real if unit == 1.0 else gS[b, kk].imag
            assert abs(fd - want) <= 1e-7 * max(1.0, abs(want))
    fd = (total(H, S, xi + h) - total(H, S, xi - h)) / (2 * h)
    assert abs(fd - gxi) <= 1e-7 * max(1.0, abs(gxi))


def test_rzf_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(28)
    nt, k, lam = 48, 6, 0.1
    H, vs, vl, xi = random_problem(rng, nt, k)
    S = qpsk(rng, (3, k))
    mask = torch.tensor(np.abs(H) > 0)
    Ht = torch.tensor(H, requires_grad=True)
    St = torch.tensor(S, requires_grad=True)
    xit = torch.tensor(xi, dtype=torch.float64, requires_grad=True)
    Hm = Ht * mask
    M = Hm @ Hm.conj().T + xit * torch.eye(k, dtype=torch.complex128)
    V = torch.linalg.solve(M, St.T)
    X = (Hm.conj().T @ V).T
    R = X @ Hm.T - St
    L = (R.abs().pow(2).sum() + lam * X.abs().pow(2).sum()) / 3
    L.backward()
    Xn, _ = oracle.rzf(H, vs, vl, S, xi)
    _, G, gHe, gSe = _loss_and_explicit(H, S, Xn, lam)
    gH, gS, gxi = oracle.rzf_grad(H, vs, vl, S, xi, G)
    np.testing.assert_allclose(gH + gHe * (np.abs(H) > 0), Ht.grad.numpy(), atol=1e-12)
    np.testing.assert_allclose(gS + gSe, St.grad.numpy(), atol=1e-12)
    assert abs(gxi - float(xit.grad)) <= 1e-12 * max(1.0, abs(gxi))


# ---------------------------------------------------------------------------
# Precoding matrix and link metrics (signal model / spectral efficiency of
# Sec. II, RZF precoder and power budget, Remark 1, NMSE of Sec. VII)
# ---------------------------------------------------------------------------

def test_single_user_rate_is_mrt_capacity():
    # K = 1: F = h / (|h|^2 + xi), so beta^2 |h^H f|^2 = |h|^2 and the rate
    # is log2(1 + |h|^2 / xi) (SNR |h|^2 rho / sigma^2)
    rng = np.random.default_rng(51)
    H, vs, vl, _ = random_problem(rng, 48, 1)
    xi = 0.37
    X = oracle.precoder(H, vs, vl, xi)
    E, beta, rate = oracle.link_metrics(H, vs, vl, xi, X)
    h2 = float(np.sum(np.abs(H[0, vs[0]:vs[0] + vl[0]]) ** 2))
    assert abs(beta - (h2 + xi) / np.sqrt(h2)) <= 1e-12 * beta
    assert abs(E[0, 0] - h2 / (h2 + xi)) <= 1e-13
    assert abs(rate[0] - np.log2(1 + h2 / xi)) <= 1e-12


def test_disjoint_vrs_no_interference():
    # users with disjoint VRs are orthogonal: M is diagonal, E is diagonal
    # with E_kk = |h_k|^2 / (|h_k|^2 + xi), and each rate has no interference
    rng = np.random.default_rng(52)
    H, vs, vl, _ = random_problem(rng, 96, 6, disjoint=True)
    xi = 0.8
    X = oracle.precoder(H, vs, vl, xi)
    E, beta, rate = oracle.link_metrics(H, vs, vl, xi, X)
    h2 = np.array([np.sum(np.abs(H[k, vs[k]:vs[k] + vl[k]]) ** 2) for k in range(6)])
    ekk = h2 / (h2 + xi)
    assert np.max(np.abs(E - np.diag(ekk))) <= 1e-13
    b2 = 1.0 / np.sum(h2 / (h2 + xi) ** 2)          # ||f_k||^2 = |h_k|^2 / (|h_k|^2 + xi)^2
    assert abs(beta ** 2 - b2) <= 1e-12 * b2
    assert np.max(np.abs(rate - np.log2(1 + b2 * ekk ** 2 / xi))) <= 1e-12


def test_effective_channel_identity_and_power_budget():
    # H F = H H^H (H H^H + xi I)^-1 = I - xi M^-1, with M formed densely and
    # inverted by LAPACK (an independent route); ||beta F||_F = 1
    rng = np.random.default_rng(53)
    H, vs, vl, _ = random_problem(rng, 80, 12)
    xi = 0.45
    Hb = oracle.band_channel(H, vs, vl)
    X = oracle.precoder(H, vs, vl, xi)
    E, beta, _ = oracle.link_metrics(H, vs, vl, xi, X)
    M = Hb @ Hb.conj().T + xi * np.eye(12)
    ref = np.eye(12) - xi * np.linalg.inv(M)
    assert np.max(np.abs(E - ref)) <= 1e-12
    assert abs(np.linalg.norm(beta * X) - 1.0) <= 1e-13
    # entries outside the VRs never enter E
    Hn = H.copy()
    for k in range(12):
        Hn[k, :vs[k]] = 5.0
        Hn[k, vs[k] + vl[k]:] = -3.0j
    E2, _, _ = oracle.link_metrics(Hn, vs, vl, xi, X)
    assert np.array_equal(E, E2)


def test_rates_invariant_under_channel_and_noise_scaling():
    # (H, xi) -> (c H, c^2 xi): M scales by c^2, F by 1/c, beta by c, E is
    # unchanged, and every SINR (signal and interference both scaled by
    # beta^2 against xi) is unchanged; with interference present this fails if
    # beta^2 or xi enters the denominator wrongly
    rng = np.random.default_rng(54)
    H, vs, vl, _ = random_problem(rng, 64, 10)
    xi, c = 0.6, 3.7
    r1 = oracle.link_metrics(H, vs, vl, xi, oracle.precoder(H, vs, vl, xi))
    r2 = oracle.link_metrics(c * H, vs, vl, c * c * xi, oracle.precoder(c * H, vs, vl, c * c * xi))
    a2 = np.abs(r1[0]) ** 2
    assert np.min(a2.sum(axis=1) - np.diag(a2)) > 1e-6          # interference is present
    assert np.max(np.abs(r1[0] - r2[0])) <= 1e-12
    assert abs(r2[1] - c * r1[1]) <= 1e-12 * r2[1]
    assert np.max(np.abs(r1[2] - r2[2])) <= 1e-12


def test_nmse_definition():
    rng = np.random.default_rng(55)
    F = rng.standard_normal((5, 9)) + 1j * rng.standard_normal((5, 9))
    assert oracle.nmse(F, F) == 0.0
    assert abs(oracle.nmse(F, 2 * F) - 1.0) <= 1e-15
    assert abs(oracle.nmse(F, F * (1 + 1e-3j)) - 1e-3) <= 1e-15


def test_interference_is_what_user_u_receives():
    # any precoder: user 1 hears stream 0 (f_0 reaches into user 1's VR), user 0
    # hears nothing of stream 1; y_u = h_u^H F s, so the interference at user u
    # is sum_{b != u} |h_u^H f_b|^2 (row u of E), not column u
    Nt, xi = 16, 0.25
    vs, vl = np.array([0, 8]), np.array([8, 8])
    H = np.zeros((2, Nt), dtype=np.complex128)
    H[0, 0:8] = 0.5
    H[1, 8:16] = 0.5j
    X = np.zeros((2, Nt), dtype=np.complex128)
    X[0, 0:8] = 1.0
    X[0, 8:10] = 0.3
    X[1, 8:16] = -1.0j
    E, beta, rate = oracle.link_metrics(H, vs, vl, xi, X)
    b2 = 1.0 / (8 + 2 * 0.09 + 8)
    e00, e10, e11 = 4.0, 0.5j * 0.3 * 2, 0.5j * -1.0j * 8
    assert np.allclose(E, [[e00, 0.0], [e10, e11]], atol=1e-15)
    assert abs(beta ** 2 - b2) <= 1e-15
    assert abs(rate[0] - np.log2(1 + b2 * 16 / xi)) <= 1e-12
    assert abs(rate[1] - np.log2(1 + b2 * abs(e11) ** 2 / (b2 * abs(e10) ** 2 + xi))) <= 1e-12


# ---------------------------------------------------------------------------
# Subarray VR model (Sec. II) and the orthogonal set on a general VR graph
# (Sec. V-B)
# ---------------------------------------------------------------------------

def _brute_mis(adj):
    K = adj.shape[0]
    best = 0
    for m in range(1 << K):
        ids = [i for i in range(K) if (m >> i) & 1]
        if all(not adj[a, b] for a in ids for b in ids):
            best = max(best, len(ids))
    return best


def _graph_as_masks(adj):
    """Subarray masks whose VR graph is adj: one subarray per edge (and
    one private subarray per vertex with no edge, so every VR is nonempty
    except where noted). Returns (masks, n_sub, nt, vs, vl, H=0)."""
    K = adj.shape[0]
    edges = [(i, j) for i in range(K) for j in range(i + 1, K) if adj[i, j]]
    masks = [0] * K
    for s, (i, j) in enumerate(edges):
        masks[i] |= 1 << s
        masks[j] |= 1 << s
    n_sub = len(edges)
    for v in range(K):
        if masks[v] == 0:
            masks[v] = 1 << n_sub
            n_sub += 1
    n_sub = max(n_sub, 1)
    assert n_sub <= 64
    nt = 2 * n_sub
    vs, vl = synth.mask_hulls(masks, nt, n_sub)
    return np.array(masks, dtype=np.uint64), n_sub, nt, vs, vl, np.zeros((K, nt), complex)


def _f_of_graph(adj):
    masks, n_sub, nt, vs, vl, H = _graph_as_masks(adj)
    assert np.array_equal(oracle.mask_graph(masks), adj)
    return oracle.mis(H, vs, vl, 1.0, masks=masks, n_sub=n_sub)


def _random_forest(rng, K):
    adj = np.zeros((K, K), dtype=bool)
    for v in range(1, K):
        if rng.random() < 0.8:
            u = int(rng.integers(0, v))
            adj[u, v] = adj[v, u] = True
    return adj


def test_reducing_peeling_exact_on_forests_and_maximal_on_graphs():
    rng = np.random.default_rng(61)
    for _ in range(40):
        K = int(rng.integers(1, 14))
        adj = _random_forest(rng, K)
        F = _f_of_graph(adj)
        assert not np.any(adj[np.ix_(F, F)])
        assert F.sum() == _brute_mis(adj)          # degree-0/1 reductions are exact on forests
    for _ in range(40):
        K = int(rng.integers(2, 11))
        while True:
            a = np.triu(rng.random((K, K)) < rng.uniform(0.1, 0.8), 1)
            if a.sum() <= 60:
                break
        adj = a | a.T
        F = _f_of_graph(adj)
        assert not np.any(adj[np.ix_(F, F)])          # independent
        for v in np.flatnonzero(~F):                  # maximal
            assert np.any(adj[v, F])
        assert F.sum() <= _brute_mis(adj)


def test_reducing_peeling_small_cases():
    # a 5-cycle has no vertex of degree <= 1: one peel, then a path of 4
    # (independence number 2); a triangle with a pendant vertex keeps the
    # pendant vertex and one far corner; a star keeps all leaves
    c5 = np.zeros((5, 5), bool)
    for i in range(5):
        c5[i, (i + 1) % 5] = c5[(i + 1) % 5, i] = True
    F = _f_of_graph(c5)
    assert F.sum() == 2 and not np.any(c5[np.ix_(F, F)])
    tri = np.zeros((4, 4), bool)
    for i, j in [(0, 1), (1, 2), (0, 2), (2, 3)]:
        tri[i, j] = tri[j, i] = True
    assert np.array_equal(_f_of_graph(tri), [True, False, False, True])
    star = np.zeros((6, 6), bool)
    star[0, 1:] = star[1:, 0] = True
    assert np.array_equal(_f_of_graph(star), [False] + [True] * 5)
    # bowtie (two triangles sharing vertex 0): no vertex of degree <= 1, so
    # the centre (largest degree) is peeled first, then the two edges reduce
    # by degree 1 to {1, 3}; peeling a smallest-degree vertex would give {2, 3}
    bow = np.zeros((5, 5), bool)
    for i, j in [(0, 1), (1, 2), (0, 2), (0, 3), (3, 4), (0, 4)]:
        bow[i, j] = bow[j, i] = True
    assert np.array_equal(_f_of_graph(bow), [False, True, False, True, False])


def test_subarray_graph_matches_antenna_indicators():
    # the subarray-level edge rule |M_i cap M_j| > 0 equals overlap of the
    # antenna-level indicator vectors u_i, u_j; users with no visible
    # subarray overlap nobody and are always in F
    rng = np.random.default_rng(62)
    nt, S, K = 120, 12, 9
    masks = np.array([sum(1 << s for s in range(S) if rng.random() < 0.35) for _ in range(K)],
                     dtype=np.uint64)
    masks[0] = 0
    U = oracle.mask_indicator(masks, nt, S)
    vs, vl = synth.mask_hulls(masks, nt, S)
    H = np.zeros((K, nt), complex)
    sets = oracle.overlap_sets(H, vs, vl, 1.0, masks=masks, n_sub=S)
    ov = (U.astype(int) @ U.T.astype(int)) > 0
    for k in range(K):
        want = sorted(set(np.flatnonzero(ov[k]).tolist()) | {k})
        assert sets[k].tolist() == want
    F = oracle.mis(H, vs, vl, 1.0, masks=masks, n_sub=S)
    assert F[0]
    assert not np.any((ov & ~np.eye(K, dtype=bool))[np.ix_(F, F)])
    for k in range(K):
        idx = np.flatnonzero(U[k])
        if idx.size == 0:
            assert vl[k] == 0
        else:
            assert vs[k] == idx[0] and vs[k] + vl[k] == idx[-1] + 1


def _masked_drop(seed, nt=96, S=8, K=7, p=0.4):
    rng = np.random.default_rng(seed)
    masks = np.array([sum(1 << s for s in range(S) if rng.random() < p) or (1 << k % S)
                      for k in range(K)], dtype=np.uint64)
    U = oracle.mask_indicator(masks, nt, S)
    Hbar = rng.standard_normal((K, nt)) + 1j * rng.standard_normal((K, nt))
    vs, vl = synth.mask_hulls(masks, nt, S)
    return masks, S, U, Hbar, vs, vl, rng


def test_masked_oracle_reads_only_visible_antennas():
    # with masks the oracle works on h_k = hbar_k * u_k (channel equation
    # with the subarray indicator): the hidden entries of Hbar are never
    # read, and the result is the dense RZF of Hbar * U, the same as the
    # hull-band model given zero gaps
    masks, S, U, Hbar, vs, vl, rng = _masked_drop(63)
    K, nt = Hbar.shape
    xi = 0.7
    Hm = Hbar * U
    Sm = rng.standard_normal((3, K)) + 1j * rng.standard_normal((3, K))
    X, V = oracle.rzf(Hbar, vs, vl, Sm, xi, masks=masks, n_sub=S)
    M = Hm @ Hm.conj().T + xi * np.eye(K)
    Vd = np.linalg.solve(M, Sm.T).T
    Xd = Vd @ Hm.conj()
    assert np.max(np.abs(X - Xd)) <= 1e-12 * np.max(np.abs(Xd))
    assert np.max(np.abs(V - Vd)) <= 1e-12 * np.max(np.abs(Vd))
    X2, _ = oracle.rzf(Hm, vs, vl, Sm, xi)
    assert np.max(np.abs(X2 - Xd)) <= 1e-12 * np.max(np.abs(Xd))
    for variant in ("vr_oahk", "vr_ogrk", "ahk", "grk"):
        out = oracle.solve(Hbar, vs, vl, Sm[0], xi, variant=variant, tol=1e-11,
                           masks=masks, n_sub=S)
        assert out["flags"] & oracle.F_CONVERGED
        assert np.max(np.abs(out["x"] - Xd[0])) <= 1e-9 * np.max(np.abs(Xd[0]))
        assert np.all(out["x"][U.sum(axis=0) == 0] == 0)   # antennas no user sees stay 0


def test_masked_gradient_is_dense_gradient_on_visible_entries():
    # dL/dH of the subarray model = the dense model's gradient at H = Hbar * U
    # on the visible entries, zero on the hidden ones (chain rule of the
    # fixed indicator)
    masks, S, U, Hbar, vs, vl, rng = _masked_drop(64)
    K, nt = Hbar.shape
    Sm = rng.standard_normal((2, K)) + 1j * rng.standard_normal((2, K))
    G = rng.standard_normal((2, nt)) + 1j * rng.standard_normal((2, nt))
    gH, gS, gxi = oracle.rzf_grad(Hbar, vs, vl, Sm, 0.9, G, masks=masks, n_sub=S)
    full = np.zeros(K, np.int32), np.full(K, nt, np.int32)
    dH, dS, dxi = oracle.rzf_grad(Hbar * U, *full, Sm, 0.9, G)
    assert np.max(np.abs(gH - dH * U)) <= 1e-12 * np.max(np.abs(dH))
    assert np.max(np.abs(gS - dS)) <= 1e-12 * np.max(np.abs(dS))
    assert abs(gxi - dxi) <= 1e-12 * abs(dxi)


def test_masked_orthogonal_step_is_sequential_projection():
    # Proposition 1 under the subarray model: users of F with disjoint masks
    # have orthogonal rows even where their hulls overlap, so the one-shot
    # step over F equals projecting onto its rows one after another
    masks, S, U, Hbar, vs, vl, rng = _masked_drop(65, K=9, p=0.25)
    K, nt = Hbar.shape
    kw = dict(masks=masks, n_sub=S)
    F = oracle.mis(Hbar, vs, vl, 0.5, **kw)
    assert F.sum() >= 2
    s = rng.standard_normal(K) + 1j * rng.standard_normal(K)
    x0 = rng.standard_normal(nt) + 1j * rng.standard_normal(nt)
    q0 = rng.standard_normal(K) + 1j * rng.standard_normal(K)
    x1, q1 = oracle.step_orthogonal(Hbar, vs, vl, 0.5, F, s, x0, q0, **kw)
    x2, q2 = x0.copy(), q0.copy()
    for i in np.flatnonzero(F):
        x2, q2 = oracle.step_row(Hbar, vs, vl, 0.5, i, s, x2, q2, **kw)
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x2))
    assert np.max(np.abs(q1 - q2)) <= 1e-12 * np.max(np.abs(q2))


def test_masked_oracle_rejects_wrong_hulls():
    masks, S, U, Hbar, vs, vl, rng = _masked_drop(66)
    bad = vs.copy()
    bad[np.argmax(vl)] += 1
    with pytest.raises(ValueError):
        oracle.rzf(Hbar, bad, vl, np.ones((1, Hbar.shape[0])), 1.0, masks=masks, n_sub=S)
    with pytest.raises(ValueError):
        oracle.mis(Hbar, vs, vl, 1.0, masks=masks, n_sub=7)   # 96 % 7 != 0
