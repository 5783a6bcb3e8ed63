"""Batching on the GPU: persistent per-XCD work queues, HIP-graph capture
and replay, the full uneven-drop workload in one launch, and the
autotuner."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel_err_rows, run_plan

pytestmark = pytest.mark.gpu


def _drops(n, nrhs, seed=None):
    return [(d.H, d.vr_start, d.vr_len, d.S, d.xi)
            for d in synth.make_workload("uneven", drops=n, nrhs=nrhs, seed=seed)]


@pytest.mark.parametrize("variant", ["vr_oahk", "grk"])
def test_persistent_equals_per_tile_launch_bitwise(variant):
    drops = _drops(12, 40)
    a, pa = run_plan(drops, variant=variant, engine="mfma", persistent=0)
    b, pb = run_plan(drops, variant=variant, engine="mfma", persistent=1)
    info = pb.query(0, 5)
    assert info[4] == 1 and info[5] <= sum(-(-d[3].shape[0] // 16) for d in drops)
    for x, y in zip(a, b):
        assert np.array_equal(x["X"], y["X"])
        assert np.array_equal(x["iters"], y["iters"])


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_capture_replays_match_eager(persistent):
    """The fwd solve + adjoint of an uneven batch captured once into a HIP
    graph and replayed with new symbols each time; every replay is checked
    against an eager run on the same inputs."""
    import torch
    from paper_2501_10689_amd import vrk
    ds = synth.make_workload("uneven", drops=5, nrhs=32, seed=7)
    specs, Ss, Gs = [], [], []
    for d in ds:
        H = torch.tensor(d.H, dtype=torch.complex64, device="cuda")
        S = torch.tensor(d.S, dtype=torch.complex64, device="cuda")
        X = torch.zeros((d.nrhs, d.nt), dtype=torch.complex64, device="cuda")
        V = torch.zeros((d.nrhs, d.k), dtype=torch.complex64, device="cuda")
        GX = torch.zeros_like(X)
        sp = vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S, X, V, GX, torch.zeros_like(H),
                             torch.zeros_like(S), torch.zeros(1, dtype=torch.float64, device="cuda"))
        specs.append(sp)
    plan = vrk.Plan(specs, vrk.options(variant="vr_oahk", engine="mfma", persistent=persistent))
    rng = np.random.default_rng(0)

    def new_inputs():
        ins = []
        for sp, d in zip(specs, ds):
            s = synth.qpsk(rng, (d.nrhs, d.k))
            gx = (rng.standard_normal((d.nrhs, d.nt)) + 1j * rng.standard_normal((d.nrhs, d.nt))) * 0.01
            ins.append((s, gx))
        return ins

    def load(ins):
        for sp, (s, gx) in zip(specs, ins):
            sp.S.copy_(torch.tensor(s, dtype=torch.complex64))
            sp.GX.copy_(torch.tensor(gx, dtype=torch.complex64))

    def outputs():
        return [(sp.X.cpu().numpy(), sp.GH.cpu().numpy(), sp.GS.cpu().numpy(), float(sp.gxi.cpu()[0]))
                for sp in specs]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.solve(stream=side)
        plan.solve_adjoint(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve()
        plan.solve_adjoint()
    torch.cuda.synchronize()
    for rep in range(4):
        ins = new_inputs()
        load(ins)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = outputs()
        load(ins)
        plan.solve()
        plan.solve_adjoint()
        torch.cuda.synchronize()
        want = outputs()
        for (xa, ha, sa, ga), (xb, hb, sb, gb) in zip(got, want):
            assert np.array_equal(xa, xb) and np.array_equal(ha, hb) and np.array_equal(sa, sb)
            assert ga == gb
        for sp, d, (s, _) in zip(specs, ds, ins):
            Xr, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, s, d.xi)
            assert rel_err_rows(sp.X.cpu().numpy().astype(np.complex128), Xr).max() <= 1e-4


def test_full_uneven_workload_one_persistent_launch():
    """512 drops (Nt in {512, 1024, 2048}, K in [16, 128], VR U[Nt/8, Nt/2],
    256 QPSK vectors each, SNR U[0, 20] dB): one persistent launch; every
    one of the 131072 vectors against the FP64 Cholesky RZF."""
    ds = synth.make_workload("uneven")
    drops = [(d.H, d.vr_start, d.vr_len, d.S, d.xi) for d in ds]
    res, plan = run_plan(drops, variant="vr_oahk", engine="mfma", persistent=1)
    worst = 0.0
    for jd, (H, vs, vl, S, xi) in enumerate(drops):
        X, _ = oracle.rzf(H, vs, vl, S, xi)
        assert np.all(res[jd]["flags"] == oracle.F_CONVERGED), jd
        worst = max(worst, rel_err_rows(res[jd]["X"], X).max())
    print("uneven workload: worst rel err %.2e" % worst)
    assert worst <= 1e-4


def test_autotune_picks_a_valid_config_and_caches(tmp_path):
    import torch
    from paper_2501_10689_amd import vrk
    ds = synth.make_workload("uneven", drops=4, nrhs=48, seed=11)
    specs = []
    for d in ds:
        specs.append(vrk.ProblemSpec(torch.tensor(d.H, dtype=torch.complex64, device="cuda"), d.vr_start,
                                     d.vr_len, d.xi, torch.tensor(d.S, dtype=torch.complex64, device="cuda"),
                                     torch.zeros((d.nrhs, d.nt), dtype=torch.complex64, device="cuda"),
                                     torch.zeros((d.nrhs, d.k), dtype=torch.complex64, device="cuda")))
    cache = str(tmp_path / "tune.txt")
    o, ms = vrk.autotune(specs, vrk.options(variant="vr_oahk"), cache_path=cache, reps=2)
    assert ms > 0 and o.engine in (1, 2)
    assert os.path.exists(cache) and len(open(cache).read().splitlines()) == 1
    o2, ms2 = vrk.autotune(specs, vrk.options(variant="vr_oahk"), cache_path=cache, reps=2)
    assert (o2.engine, o2.tile_waves, o2.persistent, o2.schedule) == (o.engine, o.tile_waves, o.persistent,
                                                                       o.schedule)
    assert abs(ms2 - ms) < 1e-3
    plan = vrk.Plan(specs, o)
    plan.solve()
    torch.cuda.synchronize()
    for sp, d in zip(specs, ds):
        Xr, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
        assert rel_err_rows(sp.X.cpu().numpy().astype(np.complex128), Xr).max() <= 1e-4


def test_binding_rejects_mismatched_buffers():
    """Host-side checks of the Python binding (nothing is launched): element
    type against the plan's, shapes against H and S, unit inner stride, the
    VR arrays' length; KaczmarzRZF rejects S of another dtype than H."""
    import torch
    from paper_2501_10689_amd import vrk
    from paper_2501_10689_amd.autograd import rzf_precode
    K, N, B = 4, 64, 3
    H = torch.zeros((K, N), dtype=torch.complex64, device="cuda")
    S = torch.zeros((B, K), dtype=torch.complex64, device="cuda")
    X = torch.zeros((B, N), dtype=torch.complex64, device="cuda")
    vs, vl = np.zeros(K, np.int32), np.full(K, 8, np.int32)
    bad = [
        dict(S=S.to(torch.complex128)),                                   # dtype
        dict(X=torch.zeros((B, N + 1), dtype=torch.complex64, device="cuda")),   # shape
        dict(X=torch.zeros((N, B), dtype=torch.complex64, device="cuda").t()),   # inner stride
        dict(GX=X, GH=torch.zeros((K, N), dtype=torch.complex64, device="cuda"),
             GS=torch.zeros((B, K + 1), dtype=torch.complex64, device="cuda"),
             gxi=torch.zeros(1, dtype=torch.float64, device="cuda")),     # GS shape
        dict(vr_len=np.full(K + 1, 8, np.int32)),                         # VR arrays
    ]
    for kw in bad:
        args = dict(H=H, vr_start=vs, vr_len=vl, xi=1.0, S=S, X=X)
        args.update(kw)
        with pytest.raises(ValueError):
            vrk.Plan([vrk.ProblemSpec(**args)], vrk.options(dtype="c64"))
    with pytest.raises(ValueError):
        rzf_precode(H, S.to(torch.complex128), 1.0, vs, vl)


@pytest.mark.parametrize("engine", ["mfma", "vector"])
def test_refresh_after_the_channel_changes(engine):
    """vrk_plan_refresh after H is overwritten in place (same VRs) gives
    the solve and gradients of a plan bound to the new channel, bit for bit,
    eagerly and as replays of a captured graph of refresh + solve + adjoint."""
    import torch
    from paper_2501_10689_amd import vrk
    ds = synth.make_workload("uneven", drops=3, nrhs=40, seed=21)
    rng = np.random.default_rng(4)
    cdt = torch.complex64

    def specs_for(Hs):
        out = []
        for d, H in zip(ds, Hs):
            Sd = torch.from_numpy(d.S).to(device="cuda", dtype=cdt)
            G = torch.from_numpy((rng.standard_normal((d.nrhs, d.nt)) + 0j) / d.nrhs).to(device="cuda", dtype=cdt)
            out.append(vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, Sd,
                                       torch.zeros((d.nrhs, d.nt), dtype=cdt, device="cuda"),
                                       torch.zeros((d.nrhs, d.k), dtype=cdt, device="cuda"), G,
                                       torch.zeros_like(H), torch.zeros_like(Sd),
                                       torch.zeros(1, dtype=torch.float64, device="cuda")))
        return out

    H0 = [torch.from_numpy(d.H).to(device="cuda", dtype=cdt) for d in ds]
    H1 = []
    for d in ds:   # another channel on the same VRs
        band = np.abs(d.H) > 0
        Hn = np.where(band, d.H * np.exp(1j * rng.uniform(0, 2 * np.pi, d.H.shape)) * 1.3, 0)
        H1.append(torch.from_numpy(Hn).to(device="cuda", dtype=cdt))
    opts = vrk.options(variant="vr_oahk", engine=engine, tol=1e-6)
    sp = specs_for([h.clone() for h in H0])
    plan = vrk.Plan(sp, opts)
    plan.solve()
    for s_, h in zip(sp, H1):
        s_.H.copy_(h)
    plan.refresh()
    plan.solve()
    plan.solve_adjoint()
    ref_sp = specs_for(H1)
    for a, b in zip(sp, ref_sp):
        b.GX.copy_(a.GX)
    ref = vrk.Plan(ref_sp, opts)
    ref.solve()
    ref.solve_adjoint()
    torch.cuda.synchronize()
    for a, b in zip(sp, ref_sp):
        for name in ("X", "V", "GH", "GS", "gxi"):
            assert torch.equal(getattr(a, name), getattr(b, name)), name
    want = [(a.X.clone(), a.GH.clone()) for a in sp]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.refresh()
        plan.solve()
        plan.solve_adjoint()
    for _ in range(3):
        for a in sp:
            a.X.zero_()
            a.GH.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, (x, gh) in zip(sp, want):
            assert torch.equal(a.X, x) and torch.equal(a.GH, gh)


@pytest.mark.parametrize("engine,variant,wave_tiles", [("vector", "vr_oahk", 0), ("vector", "grk", 0),
                                                      ("mfma", "vr_oahk", -1), ("mfma", "grk", -1),
                                                      ("mfma", "ahk", 2)])
def test_check_every(engine, variant, wave_tiles):
    """The stop rule tested every third iteration: every column still meets
    the tolerance and the RZF, its count is a multiple of three (on the
    vector engine the first multiple at or past the every-iteration count),
    and check_every 1 is the default behaviour bit for bit."""
    d = synth.make_workload("many_rhs", nrhs=35, nt=512, k=40)[0]
    drop = [(d.H, d.vr_start, d.vr_len, d.S, d.xi)]
    X, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    base, _ = run_plan(drop, variant=variant, engine=engine, tol=1e-5, wave_tiles=wave_tiles)
    from paper_2501_10689_amd import vrk
    import torch
    sp = vrk.ProblemSpec(torch.from_numpy(d.H).to("cuda", torch.complex64), d.vr_start, d.vr_len, d.xi,
                         torch.from_numpy(d.S).to("cuda", torch.complex64),
                         torch.zeros((35, 512), dtype=torch.complex64, device="cuda"),
                         torch.zeros((35, 40), dtype=torch.complex64, device="cuda"))
    for ce in (1, 3):
        plan = vrk.Plan([sp], vrk.options(variant=variant, engine=engine, tol=1e-5, wave_tiles=wave_tiles,
                                          check_every=ce))
        st = plan.stats_buffers()
        plan.solve(stats=st)
        torch.cuda.synchronize()
        it, rel, fl = [t.cpu().numpy() for t in st]
        Xg = sp.X.cpu().numpy().astype(np.complex128)
        assert np.all(fl == oracle.F_CONVERGED) and np.all(rel <= 1e-5)
        assert rel_err_rows(Xg, X).max() <= 1e-4
        if ce == 1:
            assert np.array_equal(Xg, base[0]["X"]) and np.array_equal(it, base[0]["iters"])
        else:
            assert np.all(it % 3 == 0)
            if engine == "vector":   # the first multiple of 3 at or past the every-iteration stop
                assert np.all(it >= base[0]["iters"])
            else:                    # the MFMA engines' confirm pass may end a column earlier or later
                assert abs(it.mean() - base[0]["iters"].mean()) <= 3.0
