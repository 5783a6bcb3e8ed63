"""Helpers for the GPU tests: move numpy inputs to the device and run the
HIP path through the C ABI (paper_2501_10689_amd.vrk)."""
from __future__ import annotations

import numpy as np


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def run_plan(drops, variant="vr_oahk", select="baiwu", dtype="c64", engine="auto", tol=1e-5,
             max_iters=100000, seed=0, schedule="auto", adjoint_g=None, tile_waves=0,
             persistent=0, x_pad=0):
    """drops: list of (H, vs, vl, S, xi) numpy tuples, or (H, vs, vl, S, xi,
    vr_mask, n_sub) for the subarray VR model. Returns per-drop dicts with
    X, V (numpy complex128) and stats, plus the plan. x_pad > 0 gives the X
    rows a stride of Nt + x_pad (a view into a wider buffer)."""
    import torch
    from paper_2501_10689_amd import vrk
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    specs = []
    for j, dr in enumerate(drops):
        H, vs, vl, S, xi = dr[:5]
        Hd = to_dev(H, tdt)
        Sd = to_dev(np.atleast_2d(S), tdt)
        B = Sd.shape[0]
        X = torch.full((B, H.shape[1] + x_pad), float("nan"), dtype=tdt, device="cuda")[:, :H.shape[1]]
        V = torch.full((B, H.shape[0]), float("nan"), dtype=tdt, device="cuda")
        sp = vrk.ProblemSpec(Hd, vs, vl, xi, Sd, X, V)
        if len(dr) > 5:
            sp.vr_mask, sp.n_sub = dr[5], dr[6]
        if adjoint_g is not None:
            sp.GX = to_dev(adjoint_g[j], tdt)
            sp.GH = torch.zeros_like(Hd)
            sp.GS = torch.zeros_like(Sd)
            sp.gxi = torch.zeros(1, dtype=torch.float64, device="cuda")
        specs.append(sp)
    o = vrk.options(variant=variant, select=select, dtype=dtype, engine=engine, tol=tol,
                    max_iters=max_iters, seed=seed, schedule=schedule, tile_waves=tile_waves,
                    persistent=persistent)
    plan = vrk.Plan(specs, o)
    st = plan.stats_buffers()
    plan.solve(stats=st)
    out = []
    if adjoint_g is not None:
        sta = plan.stats_buffers()
        plan.solve_adjoint(stats=sta)
    torch.cuda.synchronize()
    it, rel, fl = [t.cpu().numpy() for t in st]
    base = 0
    for j, sp in enumerate(specs):
        B = sp.S.shape[0]
        d = dict(X=sp.X.cpu().numpy().astype(np.complex128), V=sp.V.cpu().numpy().astype(np.complex128),
                 iters=it[base:base + B], relres=rel[base:base + B], flags=fl[base:base + B])
        if adjoint_g is not None:
            d["GH"] = sp.GH.cpu().numpy().astype(np.complex128)
            d["GS"] = sp.GS.cpu().numpy().astype(np.complex128)
            d["gxi"] = float(sp.gxi.cpu().numpy()[0])
            d["adj_flags"] = sta[2].cpu().numpy()[base:base + B]
        out.append(d)
        base += B
    return out, plan


def rel_err_rows(X, Xref):
    num = np.linalg.norm(X - Xref, axis=1)
    den = np.maximum(np.linalg.norm(Xref, axis=1), 1e-300)
    return num / den
