"""GPU parity of the wave-owned MFMA engine (AHK and VR-OAHK: each wave of a
tile owns whole 16-user row blocks, several tiles per compute unit) against
the FP64 oracle, through the C ABI, for every tile shape it supports."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_grads, rel_err_rows, run_plan
from tests.helpers import qpsk, random_problem

pytestmark = pytest.mark.gpu

# (waves per tile, users up to): 4 row blocks per wave with 1, 2, 4 waves,
# 2 row blocks per wave with 1, 2, 4, 8 waves (the plan picks 2 blocks per
# wave when they suffice)
SHAPES = [(1, 64), (1, 32), (2, 128), (2, 64), (4, 256), (4, 128), (8, 256)]


def _drops_for(kmax, nrhs, seed):
    """A few drops with K up to kmax (ragged K and ragged tiles), Nt a few times K."""
    rng = np.random.default_rng(seed)
    out = []
    for k in sorted({kmax, max(1, kmax - 13), max(1, kmax // 2 + 3)}):
        nt = int(rng.choice([k * 3 + 5, k * 4, 512]))
        H, vs, vl, xi = random_problem(rng, nt, k, lo=max(1, nt // 10), hi=max(2, nt // 3))
        out.append((H, vs, vl, qpsk(rng, (nrhs, k)), xi))
    return out


@pytest.mark.parametrize("waves,kmax", SHAPES)
@pytest.mark.parametrize("variant", ["ahk", "vr_oahk"])
def test_wave_tiles_match_rzf(variant, waves, kmax):
    drops = _drops_for(kmax, 37, seed=waves * 100 + kmax)
    res, plan = run_plan(drops, variant=variant, engine="mfma", tol=1e-6, wave_tiles=waves)
    eng = plan.query(0, 5)
    assert eng[10] == waves and eng[11] == (2 if kmax <= 32 * waves else 4)
    for jd, (H, vs, vl, S, xi) in enumerate(drops):
        X, V = oracle.rzf(H, vs, vl, S, xi)
        g = res[jd]
        assert np.all(g["flags"] == oracle.F_CONVERGED), (jd, g["flags"])
        assert rel_err_rows(g["X"], X).max() <= 1e-4, jd
        assert rel_err_rows(g["V"], V).max() <= 1e-4, jd
        assert np.all(g["relres"] <= 1e-6)


@pytest.mark.parametrize("waves", [1, 2])
@pytest.mark.parametrize("snr", [0.0, 20.0])
def test_wave_tiles_many_rhs_snr(waves, snr):
    """Nt 1024, K 64, 4 full tiles and a ragged one at SNR 0 and 20 dB."""
    d = synth.make_workload("many_rhs", nrhs=70, snr_db=snr)[0]
    for variant in ("ahk", "vr_oahk"):
        res, _ = run_plan([(d.H, d.vr_start, d.vr_len, d.S, d.xi)], variant=variant, engine="mfma",
                          wave_tiles=waves)
        X, V = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
        assert np.all(res[0]["flags"] == oracle.F_CONVERGED)
        assert rel_err_rows(res[0]["X"], X).max() <= 1e-4
        assert rel_err_rows(res[0]["V"], V).max() <= 1e-4


@pytest.mark.parametrize("waves", [4, 8])
def test_wave_tiles_large_shape(waves):
    """Nt 4096, K 256 (VR U[256, 1024], 16-QAM), two drops of 40 vectors."""
    ds = synth.make_workload("large", drops=2, nrhs=40)
    drops = [(d.H, d.vr_start, d.vr_len, d.S, d.xi) for d in ds]
    for variant in ("vr_oahk", "ahk"):
        res, _ = run_plan(drops, variant=variant, engine="mfma", wave_tiles=waves)
        for jd, (H, vs, vl, S, xi) in enumerate(drops):
            X, _ = oracle.rzf(H, vs, vl, S, xi)
            assert np.all(res[jd]["flags"] == oracle.F_CONVERGED), (variant, jd)
            assert rel_err_rows(res[jd]["X"], X).max() <= 1e-4, (variant, jd)


@pytest.mark.parametrize("waves,kmax", SHAPES)
def test_wave_tiles_adjoint(waves, kmax):
    drops = _drops_for(kmax, 33, seed=7 + waves)
    Gs, refs = [], []
    for (H, vs, vl, S, xi) in drops:
        X, _ = oracle.rzf(H, vs, vl, S, xi)
        G = 2.0 * ((X @ H.T - S) @ H.conj() + 0.1 * X) / S.shape[0]
        Gs.append(G)
        refs.append(oracle.rzf_grad(H, vs, vl, S, xi, G))
    res, _ = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, adjoint_g=Gs, wave_tiles=waves)
    for jd, ref in enumerate(refs):
        g = res[jd]
        assert np.all(g["adj_flags"] == oracle.F_CONVERGED), jd
        check_grads(g, ref, np.abs(drops[jd][0]) > 0, 2e-4, label="wave %d drop %d" % (waves, jd))


@pytest.mark.parametrize("waves", [1, 4])
def test_wave_tiles_edge_cases(waves):
    """Zero symbol vector (0 iterations), a user with an empty VR, all users
    disjoint (F = everyone, V empty: one iteration), K = 1, K > Nt."""
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
    H4, vs4, vl4, xi4 = random_problem(rng, 40, 1)
    drops.append((H4, vs4, vl4, qpsk(rng, (5, 1)), xi4))
    H5, vs5, vl5, xi5 = random_problem(rng, 24, 40, lo=3, hi=20)
    drops.append((H5, vs5, vl5, qpsk(rng, (20, 40)), xi5))
    for variant in ("ahk", "vr_oahk"):
        res, _ = run_plan(drops, variant=variant, engine="mfma", tol=1e-6, wave_tiles=waves)
        for jd, (H, vs, vl, S, xi) in enumerate(drops):
            X, _ = oracle.rzf(H, vs, vl, S, xi)
            g = res[jd]
            assert np.all(g["flags"] == oracle.F_CONVERGED), (variant, jd, g["flags"])
            nz = np.linalg.norm(X, axis=1) > 0
            assert rel_err_rows(g["X"], X)[nz].max() <= 1e-4, (variant, jd)
        assert res[0]["iters"][1] == 0 and not res[0]["X"][1].any()
        if variant == "vr_oahk":
            assert np.all(res[1]["iters"] == 1)


def test_wave_tiles_flags():
    rng = np.random.default_rng(10)
    H, vs, vl, xi = random_problem(rng, 128, 16)
    S = qpsk(rng, (16, 16))
    res, _ = run_plan([(H, vs, vl, S, xi)], variant="ahk", engine="mfma", tol=1e-9, max_iters=2, wave_tiles=1)
    assert np.all(res[0]["flags"] == oracle.F_MAXITER) and np.all(res[0]["iters"] == 2)
    Hn = H.copy()
    Hn[3, vs[3]] = np.nan
    res, _ = run_plan([(Hn, vs, vl, S, xi)], variant="vr_oahk", engine="mfma", wave_tiles=1)
    assert np.all(res[0]["flags"] & oracle.F_NONFINITE)


def test_wave_tiles_repeat_bitwise_and_close_to_block_tiles():
    """A second solve reproduces X and the iteration counts bit for bit;
    the block-tile engine reaches the same x to within the tolerance."""
    import torch
    d = synth.make_workload("uneven", drops=3, nrhs=40, seed=13)
    drops = [(x.H, x.vr_start, x.vr_len, x.S, x.xi) for x in d]
    a, plan = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, wave_tiles=2)
    st = plan.stats_buffers()
    plan.solve(stats=st)
    torch.cuda.synchronize()
    it = st[0].cpu().numpy()
    base = 0
    for j, sp in enumerate(plan.probs):
        B = sp.S.shape[0]
        assert np.array_equal(sp.X.cpu().numpy().astype(np.complex128), a[j]["X"])
        assert np.array_equal(it[base:base + B], a[j]["iters"])
        base += B
    # the summation orders differ, so near the FP32 floor (tol 1e-6) a column
    # may stop an iteration or a confirm pass apart
    b, _ = run_plan(drops, variant="vr_oahk", engine="mfma", tol=1e-6, wave_tiles=-1)
    for x, y in zip(a, b):
        assert rel_err_rows(x["X"], y["X"]).max() <= 2e-5
        assert np.abs(x["iters"].astype(int) - y["iters"].astype(int)).max() <= 4
        assert abs(x["iters"].mean() - y["iters"].mean()) <= 0.5
