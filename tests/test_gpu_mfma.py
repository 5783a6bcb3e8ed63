"""GPU parity of the MFMA engine (16 RHS per workgroup, FP32 matrix cores)
against the FP64 oracle, through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_grads, rel_err_rows, run_plan
from tests.helpers import qpsk, random_problem

pytestmark = pytest.mark.gpu

VARIANTS = ["grk", "ahk", "vr_ogrk", "vr_oahk"]


@pytest.mark.parametrize("snr", [0.0, 10.0, 20.0])
@pytest.mark.parametrize("waves", [8, 16])
@pytest.mark.parametrize("variant", VARIANTS)
def test_many_rhs_ragged_tiles(variant, waves, snr):
    """Nt 1024, K 64 with 37 vectors at SNR 0, 10 and 20 dB (the 20 dB point
    has the smallest xi, so the worst-conditioned Gram matrix): two full tiles
    of 16 and a ragged tail, with 8 and 16 waves per workgroup."""
    d = synth.make_workload("many_rhs", nrhs=37, snr_db=snr)[0]
    res, plan = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant=variant, engine="mfma",
                         tile_waves=waves)
    assert plan.query(0, 5)[0] == 2   # MFMA engine chosen
    g = res[0]
    X, V = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    err = rel_err_rows(g["X"], X)
    print(variant, "max err %.2e" % err.max(), "iters", g["iters"].min(), g["iters"].max())
    assert np.all(g["flags"] == oracle.F_CONVERGED)
    assert err.max() <= 1e-4
    assert rel_err_rows(g["V"], V).max() <= 1e-4
    assert np.all(g["relres"] <= 1e-5)


@pytest.mark.parametrize("nt,k,nrhs", [(1000, 20, 21), (200, 16, 16), (512, 37, 33), (2048, 128, 17),
                                       (64, 100, 16), (1536, 5, 48), (1001, 24, 19)])
@pytest.mark.parametrize("variant", ["grk", "vr_oahk", "ahk"])
@pytest.mark.parametrize("waves,x_pad", [(8, 0), (16, 0), (16, 3)])
def test_shapes_padding(nt, k, nrhs, variant, waves, x_pad):
    """Nt not a multiple of 16, K not a multiple of 16, K > Nt, tiny K, X
    rows not 32-byte aligned (Nt 1001, or a row stride of Nt + 3); 1, 2 or 4
    (row, column) entries per thread."""
    if -(-k // 16) * 16 > 16 * waves:
        pytest.skip("k beyond what %d waves hold" % waves)
    rng = np.random.default_rng(nt + k)
    H, vs, vl, xi = random_problem(rng, nt, k, lo=max(1, nt // 8), hi=max(1, nt // 2))
    S = qpsk(rng, (nrhs, k))
    res, plan = run_plan([(H, vs, vl, S, xi)], variant=variant, engine="mfma", tol=1e-5,
                         tile_waves=waves, x_pad=x_pad)
    kpad = -(-k // 16) * 16
    ep = 1
    while ep * 4 * waves < kpad:
        ep *= 2
    assert plan.query(0, 5)[6] == ep
    X, _ = oracle.rzf(H, vs, vl, S, xi)
    g = res[0]
    assert np.all(g["flags"] == oracle.F_CONVERGED), g["flags"]
    assert rel_err_rows(g["X"], X).max() <= 1e-4


def test_edge_cases_mfma():
    rng = np.random.default_rng(9)
    drops = []
    H, vs, vl, xi = random_problem(rng, 96, 12)
    vl[2] = 0
    H[2] = 0
    S = qpsk(rng, (18, 12))
    S[1] = 0
    drops.append((H, vs, vl, S, xi))
    H3, vs3, vl3, xi3 = random_problem(rng, 256, 8, disjoint=True)
    drops.append((H3, vs3, vl3, qpsk(rng, (16, 8)), xi3))
    for variant in VARIANTS:
        res, _ = run_plan(drops, variant=variant, engine="mfma", tol=1e-6)
        for jd, (H, vs, vl, S, xi) in enumerate(drops):
            X, _ = oracle.rzf(H, vs, vl, S, xi)
            g = res[jd]
            assert np.all(g["flags"] == oracle.F_CONVERGED), (variant, jd)
            nz = np.linalg.norm(X, axis=1) > 0
            assert rel_err_rows(g["X"], X)[nz].max() <= 1e-4, (variant, jd)
        assert res[0]["iters"][1] == 0 and not res[0]["X"][1].any()
        if variant == "vr_oahk":
            assert np.all(res[1]["iters"] == 1)


def test_flags_mfma():
    rng = np.random.default_rng(10)
    H, vs, vl, xi = random_problem(rng, 128, 16)
    S = qpsk(rng, (16, 16))
    res, _ = run_plan([(H, vs, vl, S, xi)], variant="ahk", engine="mfma", tol=1e-9, max_iters=2)
    assert np.all(res[0]["flags"] == oracle.F_MAXITER) and np.all(res[0]["iters"] == 2)
    Hn = H.copy()
    Hn[3, vs[3]] = np.nan
    res, _ = run_plan([(Hn, vs, vl, S, xi)], variant="vr_oahk", engine="mfma")
    assert np.all(res[0]["flags"] & oracle.F_NONFINITE)


def test_mfma_matches_vector_engine_iterations():
    """Both engines run the same method: aggregated variants need the same
    number of iterations (to within one, from FP32 rounding order)."""
    d = synth.make_workload("many_rhs", nrhs=32, nt=512, k=32)[0]
    for variant in ["ahk", "vr_oahk"]:
        a, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant=variant, engine="mfma")
        b, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant=variant, engine="vector")
        assert np.abs(a[0]["iters"] - b[0]["iters"]).max() <= 1
        assert rel_err_rows(a[0]["X"], b[0]["X"]).max() <= 5e-5


def test_uneven_batch_mfma():
    drops = [(d.H, d.vr_start, d.vr_len, d.S, d.xi)
             for d in synth.make_workload("uneven", drops=6, nrhs=24)]
    for variant in ["vr_oahk", "grk"]:
        res, _ = run_plan(drops, variant=variant, engine="mfma", tol=1e-5)
        for jd, (H, vs, vl, S, xi) in enumerate(drops):
            X, _ = oracle.rzf(H, vs, vl, S, xi)
            assert np.all(res[jd]["flags"] == oracle.F_CONVERGED), (variant, jd)
            assert rel_err_rows(res[jd]["X"], X).max() <= 1e-4, (variant, jd)


def test_full_size_many_rhs_every_vector():
    """The benchmarked launch: Nt 1024, K 64, 4096 vectors, VR-OAHK, SNR
    10 dB. Every one of the 4096 x is checked against the Cholesky RZF."""
    d = synth.make_workload("many_rhs")[0]
    res, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant="vr_oahk", engine="auto")
    X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    err = rel_err_rows(res[0]["X"], X)
    print("full size: max err %.2e mean iters %.2f" % (err.max(), res[0]["iters"].mean()))
    assert np.all(res[0]["flags"] == oracle.F_CONVERGED)
    assert err.max() <= 1e-4


@pytest.mark.parametrize("nt,k,nrhs", [(256, 16, 32), (1000, 40, 37), (64, 20, 16)])
def test_adjoint_mfma_matches_closed_form(nt, k, nrhs):
    """MFMA adjoint (b = H g, adjoint solve, band-tile gradient GEMM) vs the
    oracle's closed-form gradient, ragged RHS count and padded users."""
    rng = np.random.default_rng(11 + nt)
    H, vs, vl, xi = random_problem(rng, nt, k)
    S = qpsk(rng, (nrhs, k))
    X, _ = oracle.rzf(H, vs, vl, S, xi)
    G = 2.0 * ((X @ H.T - S) @ H.conj() + 0.1 * X) / nrhs
    gH, gS, gxi = oracle.rzf_grad(H, vs, vl, S, xi, G)
    res, _ = run_plan([(H, vs, vl, S, xi)], variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=[G])
    g = res[0]
    m = np.abs(H) > 0
    assert np.all(g["adj_flags"] == oracle.F_CONVERGED)
    check_grads(g, (gH, gS, gxi), m, 2e-4)


@pytest.mark.parametrize("waves", [8, 16])
def test_vr_oahk_large_orthogonal_set(waves):
    """Short VRs (8..24 antennas of 512) give |F| around 20 with V nonempty:
    the orthogonal half-step runs as a Gram product over the chunks holding
    F users instead of the per-entry F columns of M (used up to 16 users)."""
    rng = np.random.default_rng(100)
    H, vs, vl, xi = random_problem(rng, 512, 48, lo=8, hi=24)
    S = qpsk(rng, (40, 48))
    res, plan = run_plan([(H, vs, vl, S, xi)], variant="vr_oahk", engine="mfma", tol=1e-6, tile_waves=waves)
    nf = int(oracle.mis(H, vs, vl).sum())
    assert 16 < nf < 48
    assert len(plan.query(0, 1)) == nf
    X, V = oracle.rzf(H, vs, vl, S, xi)
    g = res[0]
    assert np.all(g["flags"] == oracle.F_CONVERGED)
    assert rel_err_rows(g["X"], X).max() <= 1e-4
    assert rel_err_rows(g["V"], V).max() <= 1e-4


def test_adjoint_mfma_rhs_split():
    """Enough right-hand sides that each gradient tile's RHS range is split
    over workgroups (partials reduced in a second kernel); K 72 leaves a
    user-block group with a single, padded block."""
    rng = np.random.default_rng(23)
    H, vs, vl, xi = random_problem(rng, 512, 72)
    S = qpsk(rng, (700, 72))
    X, _ = oracle.rzf(H, vs, vl, S, xi)
    G = 2.0 * ((X @ H.T - S) @ H.conj() + 0.1 * X) / 700
    gH, gS, gxi = oracle.rzf_grad(H, vs, vl, S, xi, G)
    res, plan = run_plan([(H, vs, vl, S, xi)], variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=[G])
    assert plan.query(0, 5)[7] > 1
    g = res[0]
    m = np.abs(H) > 0
    assert np.all(g["adj_flags"] == oracle.F_CONVERGED)
    check_grads(g, (gH, gS, gxi), m, 2e-4)


def test_adjoint_mfma_uneven_batch():
    """One launch of each adjoint kernel over several drops of uneven shape."""
    ds = synth.make_workload("uneven", drops=4, nrhs=20)
    drops, Gs, refs = [], [], []
    for d in ds:
        X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
        G = 2.0 * ((X @ d.H.T - d.S) @ d.H.conj() + 0.1 * X) / d.nrhs
        drops.append((d.H, d.vr_start, d.vr_len, d.S, d.xi))
        Gs.append(G)
        refs.append(oracle.rzf_grad(d.H, d.vr_start, d.vr_len, d.S, d.xi, G))
    res, _ = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=Gs)
    for jd, (gH, gS, gxi) in enumerate(refs):
        g = res[jd]
        m = np.abs(drops[jd][0]) > 0
        check_grads(g, (gH, gS, gxi), m, 2e-4, label="drop %d" % jd)


@pytest.mark.parametrize("variant", ["vr_oahk", "ahk", "grk", "vr_ogrk"])
def test_large_shape(variant):
    """Nt 4096, K 256 (VR U[256, 1024], 16-QAM): four (row, column) entries
    per thread with 16 waves; 2 drops x 40 vectors."""
    ds = synth.make_workload("large", drops=2, nrhs=40)
    drops = [(d.H, d.vr_start, d.vr_len, d.S, d.xi) for d in ds]
    res, plan = run_plan(drops, variant=variant, engine="mfma", tol=1e-5)
    assert plan.query(0, 5)[6] == 4
    for jd, (H, vs, vl, S, xi) in enumerate(drops):
        X, _ = oracle.rzf(H, vs, vl, S, xi)
        assert np.all(res[jd]["flags"] == oracle.F_CONVERGED), (variant, jd)
        assert rel_err_rows(res[jd]["X"], X).max() <= 1e-4, (variant, jd)


def test_large_shape_adjoint():
    ds = synth.make_workload("large", drops=1, nrhs=32)
    d = ds[0]
    X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    G = 2.0 * ((X @ d.H.T - d.S) @ d.H.conj() + 0.1 * X) / d.nrhs
    gH, gS, gxi = oracle.rzf_grad(d.H, d.vr_start, d.vr_len, d.S, d.xi, G)
    res, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant="vr_oahk", engine="mfma", tol=1e-6,
                      adjoint_g=[G])
    g = res[0]
    m = np.abs(d.H) > 0
    check_grads(g, (gH, gS, gxi), m, 2e-4)


@pytest.mark.parametrize("engine", ["mfma", "vector"])
def test_rebind_and_resolve_are_bitwise_deterministic(engine):
    """Binding again (row norms, tiles and Gram tiles recomputed from H) and
    solving again reproduce X, V and the iteration counts bit for bit; so
    does a second plan on the same inputs."""
    import torch
    from paper_2501_10689_amd import vrk
    d = synth.make_workload("uneven", drops=3, nrhs=40, seed=11)
    drops = [(x.H, x.vr_start, x.vr_len, x.S, x.xi) for x in d]
    a, plan = run_plan(drops, variant="vr_oahk", engine=engine, tol=1e-6)
    st = plan.stats_buffers()
    plan.bind()
    plan.solve(stats=st)
    torch.cuda.synchronize()
    it = st[0].cpu().numpy()
    base = 0
    for j, sp in enumerate(plan.probs):
        B = sp.S.shape[0]
        assert np.array_equal(sp.X.cpu().numpy().astype(np.complex128), a[j]["X"])
        assert np.array_equal(it[base:base + B], a[j]["iters"])
        base += B
    b, _ = run_plan(drops, variant="vr_oahk", engine=engine, tol=1e-6)
    for x, y in zip(a, b):
        assert np.array_equal(x["X"], y["X"]) and np.array_equal(x["V"], y["V"])


@pytest.mark.parametrize("variant", ["grk", "vr_ogrk"])
@pytest.mark.parametrize("rule", ["max", "residual", "energy", "uniform"])
def test_greedy_rules_mfma(variant, rule):
    """The greedy-Kaczmarz (max), printed residual-proportional, energy and
    uniform rules on the MFMA engine: Nt 1024, K 64, 37 vectors, every x
    within 1e-4 of the FP64 RZF. The max rule is deterministic: both greedy
    variants take the same rows, so they agree bit for bit."""
    d = synth.make_workload("many_rhs", nrhs=37)[0]
    res, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant=variant, select=rule, engine="mfma")
    X, V = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    g = res[0]
    assert np.all(g["flags"] == oracle.F_CONVERGED)
    assert rel_err_rows(g["X"], X).max() <= 1e-4
    assert rel_err_rows(g["V"], V).max() <= 1e-4
    if rule == "max":
        other = "vr_ogrk" if variant == "grk" else "grk"
        r2, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant=other, select=rule, engine="mfma")
        assert np.array_equal(r2[0]["X"], g["X"]) and np.array_equal(r2[0]["iters"], g["iters"])


def _loss_grad(d, X, n_vec):
    """Incoming gradient of L = (1/n_vec) sum ||H x - s||^2 + 0.1 ||x||^2 on
    X (2 dL/d conj x), from the oracle's X."""
    return 2.0 * ((X @ d.H.T - d.S) @ d.H.conj() + 0.1 * X) / n_vec


def test_adjoint_full_workload_reduction_runs():
    """The adjoint workload as benchmarked: 256 drops of Nt 1024, K 64 with
    64 QPSK vectors each, forward + adjoint in one launch each. The gradient
    reduction takes runs of many band tiles per workgroup here (asserted), a
    path one-drop tests never reach. Every x within 1e-4 of the FP64 RZF and
    every drop's dL/dH, dL/ds, dL/dxi against the closed form, entry by entry."""
    ds = synth.make_workload("adjoint")
    n_vec = sum(d.nrhs for d in ds)
    drops, Gs, Xs = [], [], []
    for d in ds:
        X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
        drops.append((d.H, d.vr_start, d.vr_len, d.S, d.xi))
        Gs.append(_loss_grad(d, X, n_vec))
        Xs.append(X)
    res, plan = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=Gs)
    gq = plan.query(0, 7)
    print("gradient plan: band tiles %d, splits %d, C blocks %d, runs %d, longest run %d"
          % (gq[0], gq[1], gq[2], gq[4], gq[5]))
    assert gq[5] > 1
    worst = {}
    for jd, d in enumerate(ds):
        g = res[jd]
        assert np.all(g["flags"] == oracle.F_CONVERGED) and np.all(g["adj_flags"] == oracle.F_CONVERGED), jd
        assert rel_err_rows(g["X"], Xs[jd]).max() <= 1e-4, jd
        ref = oracle.rzf_grad(d.H, d.vr_start, d.vr_len, d.S, d.xi, Gs[jd])
        r = check_grads(g, ref, np.abs(d.H) > 0, 2e-4, label="drop %d" % jd)
        worst = {k: max(v, worst.get(k, 0.0)) for k, v in r.items()}
    print("worst over drops:", worst)


def test_large_adjoint_reduction_runs():
    """Six drops of the large workload at full size (Nt 4096, K 256, VR
    U[256, 1024], 1024 16-QAM vectors each): enough band tiles that each
    reduction workgroup takes runs of two or more. Forward every x within
    1e-4, adjoint against the closed form entry by entry."""
    ds = synth.make_workload("large", drops=6)
    n_vec = sum(d.nrhs for d in ds)
    drops, Gs, Xs = [], [], []
    for d in ds:
        X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
        drops.append((d.H, d.vr_start, d.vr_len, d.S, d.xi))
        Gs.append(_loss_grad(d, X, n_vec))
        Xs.append(X)
    res, plan = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=Gs)
    gq = plan.query(0, 7)
    print("gradient plan: band tiles %d, splits %d, runs %d, longest run %d" % (gq[0], gq[1], gq[4], gq[5]))
    assert gq[5] > 1
    for jd, d in enumerate(ds):
        g = res[jd]
        assert np.all(g["flags"] == oracle.F_CONVERGED) and np.all(g["adj_flags"] == oracle.F_CONVERGED), jd
        assert rel_err_rows(g["X"], Xs[jd]).max() <= 1e-4, jd
        ref = oracle.rzf_grad(d.H, d.vr_start, d.vr_len, d.S, d.xi, Gs[jd])
        check_grads(g, ref, np.abs(d.H) > 0, 2e-4, label="large drop %d" % jd)


@pytest.mark.parametrize("nrhs", [64, 256])
def test_adjoint_band_tiles_with_gaps_in_the_block_set(nrhs):
    """VRs built so that the user blocks meeting an antenna block are not
    contiguous (Nt 1024, K 64: four blocks of 16 users in VR-start order, the
    first and third with long VRs, the second and fourth with short ones), so
    the gradient's band loop runs its variants for block sets such as {0, 2},
    {0, 2, 3} and {2} as well as {0} and {0, 1}; 64 vectors (one RHS split per
    band tile) and 256 (split tiles). dL/dH, dL/ds, dL/dxi against the closed
    form entry by entry."""
    rng = np.random.default_rng(77)
    nt, k = 1024, 64
    starts = np.concatenate([np.arange(16), 100 + np.arange(16), 200 + np.arange(16), 300 + np.arange(16)])
    lens = np.concatenate([1008 - np.arange(16), np.full(16, 60), np.full(16, 800), np.full(16, 40)])
    order = rng.permutation(k)
    vs, vl = starts[order].astype(np.int32), lens[order].astype(np.int32)
    H = np.zeros((k, nt), dtype=np.complex128)
    for u in range(k):
        H[u, vs[u]:vs[u] + vl[u]] = (rng.standard_normal(vl[u]) + 1j * rng.standard_normal(vl[u])) * 0.3
    xi = k / 10.0
    # the block sets per 16-antenna block, blocks in VR-start order
    srt = np.argsort(vs, kind="stable")
    hull = [(vs[srt[16 * b:16 * b + 16]].min(), (vs + vl)[srt[16 * b:16 * b + 16]].max()) for b in range(4)]
    sets = {tuple(b for b in range(4) if hull[b][0] < 16 * (ab + 1) and 16 * ab < hull[b][1]) for ab in range(nt // 16)}
    assert (vs + vl).max() <= nt and {(0, 2), (0, 2, 3), (2,)} <= sets, sets
    S = qpsk(rng, (nrhs, k))
    X, _ = oracle.rzf(H, vs, vl, S, xi)
    d = type("D", (), {"H": H, "S": S})
    G = _loss_grad(d, X, nrhs)
    res, plan = run_plan([(H, vs, vl, S, xi)], variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=[G])
    g = res[0]
    print("gradient plan: band tiles %d, splits %d" % tuple(plan.query(0, 7)[:2]))
    assert np.all(g["flags"] == oracle.F_CONVERGED) and np.all(g["adj_flags"] == oracle.F_CONVERGED)
    assert rel_err_rows(g["X"], X).max() <= 1e-4
    ref = oracle.rzf_grad(H, vs, vl, S, xi, G)
    check_grads(g, ref, np.abs(H) > 0, 2e-4, label="block-set gaps, %d vectors" % nrhs)


@pytest.mark.parametrize("wave_tiles", [0, 2])
def test_wide_array_many_drops(wave_tiles):
    """Thirty-two drops of Nt 8192 (512 antenna blocks: the tile packing and the
    Gram kernels search offset tables of more than 256 entries, in several
    passes) with K 48 and VR U[512, 2048], 16 QPSK vectors each: enough
    tiles that the packing takes four items per wave. VR-OAHK forward and
    adjoint on the block tiles and on wave-owned tiles; every x within 1e-4
    of the FP64 RZF and every gradient against the closed form entry by
    entry."""
    rng = np.random.default_rng(8192)
    nt, k, nv = 8192, 48, 16
    drops, Gs, Xs, ref = [], [], [], []
    for _ in range(32):
        H, vs, vl, xi = random_problem(rng, nt, k, lo=512, hi=2048)
        S = qpsk(rng, (nv, k))
        X, _ = oracle.rzf(H, vs, vl, S, xi)
        d = type("D", (), {"H": H, "S": S})
        drops.append((H, vs, vl, S, xi))
        Xs.append(X)
        Gs.append(_loss_grad(d, X, 32 * nv))
    res, plan = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=Gs, wave_tiles=wave_tiles)
    tq = [plan.query(j, 6) for j in range(len(drops))]
    # residual, aggregation and Gram tiles: enough for the four-item packing
    assert max(max(int(t[0]), int(t[1]), int(t[3])) for t in tq) * len(drops) >= 4 * 16384, tq[0]
    for jd, (H, vs, vl, S, xi) in enumerate(drops):
        g = res[jd]
        assert np.all(g["flags"] == oracle.F_CONVERGED) and np.all(g["adj_flags"] == oracle.F_CONVERGED), jd
        assert rel_err_rows(g["X"], Xs[jd]).max() <= 1e-4, jd
        r = oracle.rzf_grad(H, vs, vl, S, xi, Gs[jd])
        check_grads(g, r, np.abs(H) > 0, 2e-4, label="Nt 8192 drop %d" % jd)
