"""Subarray VR model on the GPU (Sec. II with the Bernoulli subarray
visibility of the simulation section): users see unions of subarrays, the
plan takes overlap and F from the masks (reducing-peeling), the kernels read
H on each user's hull with zero gaps. Against the FP64 oracle run on the same
masks."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_grads, rel_err_rows, run_plan

pytestmark = pytest.mark.gpu


def _drops(n, nrhs, **kw):
    return synth.make_workload("subarray", drops=n, nrhs=nrhs, **kw)


def _tuple(d):
    return (d.H, d.vr_start, d.vr_len, d.S, d.xi, d.vr_mask, d.n_sub)


def _sparse_drop(seed, nt=320, n_sub=16, k=24, p=0.2, nrhs=20):
    """A drop with sparse visibility, so that F has several users whose hulls
    overlap although their masks do not."""
    rng = np.random.default_rng(seed)
    d = synth.make_subarray_drop(rng, nt=nt, k=k, nrhs=nrhs, n_sub=n_sub, p_vis=p, snr_db=10.0,
                                 fc=28e9, r_lo=5.0)
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    F = np.flatnonzero(oracle.mis(d.H, d.vr_start, d.vr_len, d.xi, **kw))
    hull_pairs = sum(1 for a in F for b in F if a < b and d.vr_len[a] and d.vr_len[b] and
                     max(d.vr_start[a], d.vr_start[b]) <
                     min(d.vr_start[a] + d.vr_len[a], d.vr_start[b] + d.vr_len[b]))
    assert hull_pairs >= 1
    return d


@pytest.mark.parametrize("variant", ["vr_oahk", "vr_ogrk", "ahk", "grk"])
def test_subarray_mfma_matches_rzf(variant):
    # four drops of the simulation setting (Nt 2000, S 20, p 0.35, K 30,
    # SNR 0 dB), 40 vectors each (two full tiles and a ragged one)
    ds = _drops(4, 40)
    res, plan = run_plan([_tuple(d) for d in ds], variant=variant, engine="mfma", tol=1e-5)
    for j, (d, r) in enumerate(zip(ds, res)):
        kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
        X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, **kw)
        assert np.all(r["flags"] == oracle.F_CONVERGED)
        assert rel_err_rows(r["X"], X).max() <= 1e-4
        f = np.zeros(d.k, bool)
        f[plan.query(j, 1)] = True
        assert np.array_equal(f, oracle.mis(d.H, d.vr_start, d.vr_len, d.xi, **kw))
        unseen = oracle.mask_indicator(d.vr_mask, d.nt, d.n_sub).sum(axis=0) == 0
        assert np.all(r["X"][:, unseen] == 0)


@pytest.mark.parametrize("variant,schedule", [("vr_oahk", "gather"), ("vr_oahk", "colour"),
                                              ("vr_ogrk", "gather"), ("ahk", "colour")])
def test_subarray_c128_vector_follows_oracle(variant, schedule):
    # complex128 vector engine against the oracle's own iteration on the same
    # masks: same F, same rows drawn, same iteration counts, iterates equal
    # to rounding; F holds users with overlapping hulls, updated one at a time
    d = _sparse_drop(7)
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    res, _ = run_plan([_tuple(d)], variant=variant, dtype="c128", engine="vector", tol=1e-10,
                      schedule=schedule)
    r = res[0]
    for b in range(d.nrhs):
        o = oracle.solve(d.H, d.vr_start, d.vr_len, d.S[b], d.xi, variant=variant, tol=1e-10,
                         rhs=b, **kw)
        assert r["iters"][b] == o["iters"]
        assert np.max(np.abs(r["X"][b] - o["x"])) <= 1e-9 * np.max(np.abs(o["x"]))
    X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, **kw)
    assert rel_err_rows(r["X"], X).max() <= 1e-8


def test_subarray_colour_and_gather_schedules_agree():
    # complex64 vector engine: the colour schedule (greedy classes of the
    # mask graph, several users with overlapping hulls per class) and the
    # antenna-gather schedule reach the same RZF
    d = _sparse_drop(7, nrhs=24)
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, **kw)
    out = {}
    for sch in ("colour", "gather"):
        res, plan = run_plan([_tuple(d)], variant="vr_oahk", engine="vector", tol=1e-6, schedule=sch)
        assert np.all(res[0]["flags"] == oracle.F_CONVERGED)
        assert rel_err_rows(res[0]["X"], X).max() <= 1e-5
        out[sch] = res[0]["X"]
    col = plan.query(0, 2)
    vs, ve = d.vr_start, d.vr_start + d.vr_len
    assert any(col[a] == col[b] and max(vs[a], vs[b]) < min(ve[a], ve[b])
               for a in range(d.k) for b in range(a + 1, d.k))
    assert rel_err_rows(out["colour"], out["gather"]).max() <= 1e-5


@pytest.mark.parametrize("engine,dtype,tol,bound", [("mfma", "c64", 1e-6, 2e-4),
                                                    ("vector", "c128", 1e-12, 1e-9)])
def test_subarray_adjoint_matches_closed_form(engine, dtype, tol, bound):
    # GH is the gradient on the visible entries and exactly zero on the
    # hidden ones inside each hull
    d = _sparse_drop(8, nrhs=32) if engine == "vector" else _drops(1, 37)[0]
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, **kw)
    G = 2.0 * ((X @ d.H.T - d.S) @ d.H.conj() + 0.1 * X) / d.nrhs
    gH, gS, gxi = oracle.rzf_grad(d.H, d.vr_start, d.vr_len, d.S, d.xi, G, **kw)
    res, _ = run_plan([_tuple(d)], variant="vr_oahk", dtype=dtype, engine=engine, tol=tol, adjoint_g=[G])
    g = res[0]
    U = oracle.mask_indicator(d.vr_mask, d.nt, d.n_sub).astype(bool)
    assert np.all(g["adj_flags"] == oracle.F_CONVERGED)
    assert np.all(g["GH"][~U] == 0)
    check_grads(g, (gH, gS, gxi), U, bound)


def test_subarray_autograd_masks_the_channel_gradient():
    # torch autograd through h = hbar * u: the library's GH (zero on hidden
    # antennas) times the indicator is the gradient with respect to hbar
    import torch
    from paper_2501_10689_amd.autograd import rzf_precode
    d = _drops(1, 64)[0]
    U = torch.tensor(oracle.mask_indicator(d.vr_mask, d.nt, d.n_sub), device="cuda")
    rng = np.random.default_rng(9)
    Hbar = d.H + (1.0 - oracle.mask_indicator(d.vr_mask, d.nt, d.n_sub)) * (
        rng.standard_normal(d.H.shape) + 1j * rng.standard_normal(d.H.shape))
    Hb = torch.tensor(Hbar, dtype=torch.complex64, device="cuda", requires_grad=True)
    St = torch.tensor(d.S, dtype=torch.complex64, device="cuda")
    Hm = Hb * U
    X = rzf_precode(Hm, St, d.xi, d.vr_start, d.vr_len, vr_mask=d.vr_mask, n_sub=d.n_sub, tol=1e-6)
    L = (X.abs().pow(2).sum()) / d.nrhs
    L.backward()
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    Xr, _ = oracle.rzf(Hbar, d.vr_start, d.vr_len, d.S, d.xi, **kw)
    gH, _, _ = oracle.rzf_grad(Hbar, d.vr_start, d.vr_len, d.S, d.xi, 2.0 * Xr / d.nrhs, **kw)
    got = Hb.grad.cpu().numpy()
    assert np.all(got[oracle.mask_indicator(d.vr_mask, d.nt, d.n_sub) == 0] == 0)
    assert np.linalg.norm(got - gH) <= 2e-4 * np.linalg.norm(gH)
    # entry by entry and per user row, relative to the largest entry / row
    assert np.abs(got - gH).max() <= 1e-3 * np.abs(gH).max()
    assert (np.linalg.norm(got - gH, axis=1)).max() <= 1e-3 * np.linalg.norm(gH, axis=1).max()


def test_subarray_full_workload_every_vector():
    # the whole subarray workload as timed: 64 drops x 256 QPSK vectors in
    # one MFMA launch, every vector within 1e-4 of the FP64 RZF
    ds = _drops(64, 256)
    res, _ = run_plan([_tuple(d) for d in ds], variant="vr_oahk", engine="mfma", tol=1e-5)
    worst = 0.0
    for d, r in zip(ds, res):
        X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, masks=d.vr_mask, n_sub=d.n_sub)
        assert np.all(r["flags"] == oracle.F_CONVERGED)
        worst = max(worst, rel_err_rows(r["X"], X).max())
    assert worst <= 1e-4


def test_subarray_user_without_visible_subarray():
    # a user that sees no subarray: empty hull, zero channel, in F, x
    # untouched by it; its v entry is s / xi
    d = _drops(1, 24)[0]
    H, vs, vl, mask = d.H.copy(), d.vr_start.copy(), d.vr_len.copy(), d.vr_mask.copy()
    H[5] = 0
    vs[5] = vl[5] = 0
    mask[5] = 0
    res, plan = run_plan([(H, vs, vl, d.S, d.xi, mask, d.n_sub)], variant="vr_oahk", engine="mfma", tol=1e-6)
    X, V = oracle.rzf(H, vs, vl, d.S, d.xi, masks=mask, n_sub=d.n_sub)
    assert 5 in plan.query(0, 1)
    assert rel_err_rows(res[0]["X"], X).max() <= 1e-4
    assert np.max(np.abs(res[0]["V"][:, 5] - d.S[:, 5] / d.xi)) <= 1e-5 * np.max(np.abs(d.S[:, 5] / d.xi))


@pytest.mark.parametrize("nt,n_sub,k,p,engine,dtype", [
    (128, 64, 1, 1.0, "vector", "c128"),     # one user seeing every subarray (hull = array)
    (64, 64, 20, 0.3, "mfma", "c64"),        # one antenna per subarray, bit 63 in use
    (64, 64, 20, 0.3, "vector", "c128"),
    (300, 3, 40, 0.5, "mfma", "c64"),        # three wide subarrays, K > Nt / 8
])
def test_subarray_edge_shapes(nt, n_sub, k, p, engine, dtype):
    rng = np.random.default_rng(nt + n_sub + k)
    d = synth.make_subarray_drop(rng, nt=nt, k=k, nrhs=20, n_sub=n_sub, p_vis=p, snr_db=10.0, fc=28e9,
                                 r_lo=5.0)
    if k > 1:
        d.vr_mask[1] = 0
        d.H[1] = 0
        d.vr_start[1] = d.vr_len[1] = 0
        d.vr_mask[2] = np.uint64(1) << np.uint64(n_sub - 1)
        d.H[2, : nt - nt // n_sub] = 0
        d.H[2, nt - nt // n_sub:] = 1.0 + 0.5j
        d.vr_start[2], d.vr_len[2] = nt - nt // n_sub, nt // n_sub
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    X, V = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, **kw)
    tol = 1e-12 if dtype == "c128" else 1e-6
    res, plan = run_plan([_tuple(d)], variant="vr_oahk", dtype=dtype, engine=engine, tol=tol)
    r = res[0]
    assert np.all(r["flags"] == oracle.F_CONVERGED)
    assert rel_err_rows(r["X"], X).max() <= (1e-9 if dtype == "c128" else 1e-4)
    f = np.zeros(k, bool)
    f[plan.query(0, 1)] = True
    assert np.array_equal(f, oracle.mis(d.H, d.vr_start, d.vr_len, d.xi, **kw))


def test_subarray_autotune_keys_on_masks(tmp_path):
    # the autotuner times candidates on masked drops, caches the winner under
    # a key that includes the masks (other masks on the same shapes: a new
    # entry), and the tuned plan still meets the RZF
    import torch
    from paper_2501_10689_amd import vrk
    ds = _drops(3, 32)
    def specs_of(drops):
        return [vrk.ProblemSpec(torch.tensor(d.H, dtype=torch.complex64, device="cuda"), d.vr_start, d.vr_len,
                                d.xi, torch.tensor(d.S, dtype=torch.complex64, device="cuda"),
                                torch.zeros((d.nrhs, d.nt), dtype=torch.complex64, device="cuda"),
                                torch.zeros((d.nrhs, d.k), dtype=torch.complex64, device="cuda"),
                                vr_mask=d.vr_mask, n_sub=d.n_sub) for d in drops]
    specs = specs_of(ds)
    cache = str(tmp_path / "tune.txt")
    o, ms = vrk.autotune(specs, vrk.options(variant="vr_oahk"), cache_path=cache, reps=2)
    assert ms > 0 and len(open(cache).read().splitlines()) == 1
    # the same hulls with one hidden subarray made visible (its channel stays
    # zero, which is a valid input): only the masks differ
    import copy
    other = [copy.deepcopy(d) for d in ds]
    for d in other:
        for u in range(d.k):
            m = int(d.vr_mask[u])
            gaps = [s_ for s_ in range(d.n_sub) if m and (m >> s_) & 1 == 0
                    and s_ * (d.nt // d.n_sub) >= d.vr_start[u]
                    and (s_ + 1) * (d.nt // d.n_sub) <= d.vr_start[u] + d.vr_len[u]]
            if gaps:
                d.vr_mask[u] = np.uint64(m | (1 << gaps[0]))
                break
    assert any(not np.array_equal(a.vr_mask, b.vr_mask) for a, b in zip(ds, other))
    vrk.autotune(specs_of(other), vrk.options(variant="vr_oahk"), cache_path=cache, reps=2)
    assert len(open(cache).read().splitlines()) == 2
    plan = vrk.Plan(specs, o)
    plan.solve()
    torch.cuda.synchronize()
    for sp, d in zip(specs, ds):
        Xr, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, masks=d.vr_mask, n_sub=d.n_sub)
        assert rel_err_rows(sp.X.cpu().numpy().astype(np.complex128), Xr).max() <= 1e-4
