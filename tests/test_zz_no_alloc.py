"""GPU test of vrk_plan_bind_static, the binding to the library's own scratch
array (for callers that cannot allocate device memory), through the C ABI:
its solves and gradients equal those of the same plan bound to a caller
workspace with vrk_plan_bind, bit for bit (same kernels, same inputs), on two
bindings in a row, the second with a smaller problem."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.helpers import qpsk, random_problem

pytestmark = pytest.mark.gpu


def _specs(drops, adjoint, tdt):
    import torch
    from paper_2501_10689_amd import vrk
    specs = []
    for (H, vs, vl, S, xi, G) in drops:
        Hd = torch.from_numpy(H).to(device="cuda", dtype=tdt)
        Sd = torch.from_numpy(S).to(device="cuda", dtype=tdt)
        B, K, N = S.shape[0], H.shape[0], H.shape[1]
        sp = vrk.ProblemSpec(Hd, vs, vl, xi, Sd, torch.full((B, N), float("nan"), dtype=tdt, device="cuda"),
                             torch.full((B, K), float("nan"), dtype=tdt, device="cuda"))
        if adjoint:
            sp.GX = torch.from_numpy(G).to(device="cuda", dtype=tdt)
            sp.GH = torch.zeros_like(Hd)
            sp.GS = torch.zeros_like(Sd)
            sp.gxi = torch.zeros(1, dtype=torch.float64, device="cuda")
        specs.append(sp)
    return specs


def _run(drops, opts, static, adjoint, tdt):
    import torch
    from paper_2501_10689_amd import vrk
    specs = _specs(drops, adjoint, tdt)
    plan = vrk.Plan(specs, opts, static=static)
    assert (plan.workspace is None) == static
    st = plan.stats_buffers()
    plan.solve(stats=st)
    if adjoint:
        plan.solve_adjoint()
    torch.cuda.synchronize()
    out = [dict(X=sp.X.cpu().numpy(), V=sp.V.cpu().numpy()) for sp in specs]
    if adjoint:
        for o, sp in zip(out, specs):
            o.update(GH=sp.GH.cpu().numpy(), GS=sp.GS.cpu().numpy(), gxi=sp.gxi.cpu().numpy())
    return out, [t.cpu().numpy() for t in st], plan


def _drops_large():
    ds = synth.make_workload("many_rhs", nrhs=256)
    rng = np.random.default_rng(5)
    return [(d.H, d.vr_start, d.vr_len, d.S, d.xi,
             (rng.standard_normal((d.nrhs, d.nt)) + 1j * rng.standard_normal((d.nrhs, d.nt))) / d.nrhs)
            for d in ds]


def _drops_small():
    rng = np.random.default_rng(6)
    out = []
    for nt, k, b in [(300, 20, 37), (512, 33, 18)]:
        H, vs, vl, xi = random_problem(rng, nt, k)
        S = qpsk(rng, (b, k))
        G = (rng.standard_normal((b, nt)) + 1j * rng.standard_normal((b, nt))) / b
        out.append((H, vs, vl, S, xi, G))
    return out


@pytest.mark.parametrize("engine,dtype", [("mfma", "c64"), ("vector", "c64"), ("vector", "c128")])
def test_bind_static_matches_caller_workspace(engine, dtype):
    import torch
    from paper_2501_10689_amd import vrk
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    opts = vrk.options(variant="vr_oahk", dtype=dtype, engine=engine, tol=1e-6)
    plans = []
    for drops in (_drops_large(), _drops_small()):   # the second binding is the smaller one
        ref, st_ref, _ = _run(drops, opts, static=False, adjoint=True, tdt=tdt)
        got, st_got, plan = _run(drops, opts, static=True, adjoint=True, tdt=tdt)
        assert plan.ws_bytes <= vrk.SCRATCH_BYTES
        for a, b in zip(ref, got):
            for key in a:
                assert np.array_equal(a[key], b[key]), key
            assert np.isfinite(b["X"]).all()
        for a, b in zip(st_ref, st_got):
            assert np.array_equal(a, b)
        assert np.all(st_got[2] == 1)
        plans.append(plan)
    # the first plan's binding was taken over by the second: its calls are refused
    with pytest.raises(vrk.VrkError) as ei:
        plans[0].solve()
    assert ei.value.status == 5
    # bound again, it runs (and now the second plan is the stale one)
    plans[0].bind()
    plans[0].solve()
    torch.cuda.synchronize()
    with pytest.raises(vrk.VrkError) as ei:
        plans[1].solve()
    assert ei.value.status == 5


def test_bind_static_rejects_a_plan_beyond_the_scratch_size():
    import torch
    from paper_2501_10689_amd import vrk
    # twelve drops of the large workload with adjoint buffers need about 100 MiB
    d = synth.make_workload("large", drops=12, nrhs=1024)
    drops = [(x.H, x.vr_start, x.vr_len, x.S, x.xi, np.zeros((x.nrhs, x.nt))) for x in d]
    specs = _specs(drops, adjoint=True, tdt=torch.complex64)
    with pytest.raises(vrk.VrkError) as ei:
        vrk.Plan(specs, vrk.options(variant="vr_oahk"), static=True)
    assert ei.value.status == 3
    assert "scratch" in str(ei.value)
