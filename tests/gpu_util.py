"""Helpers for the GPU tests: move numpy inputs to the device and run the
HIP path through the C ABI (paper_2501_10689_amd.vrk)."""
from __future__ import annotations

import numpy as np


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def run_plan(drops, variant="vr_oahk", select="baiwu", dtype="c64", engine="auto", tol=1e-5,
             max_iters=100000, seed=0, schedule="auto", adjoint_g=None, tile_waves=0,
             persistent=0, x_pad=0, wave_tiles=0):
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
                    persistent=persistent, wave_tiles=wave_tiles)
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


def check_grads(g, ref, mask, norm_bound, entry_bound=None, label=""):
    """Gradient parity against the oracle's closed form (gH, gS, gxi) =
    ref, on the band entries `mask` of H:
      - in norm: ||dGH|| <= b ||gH||, ||dGS|| <= b ||gS||, |dgxi| <= b |gxi|
        with b = norm_bound;
      - entry by entry: |dGH[k, n]| <= e max|gH| on every band entry and
        ||dGH[k, :]|| <= e max_k ||gH[k, :]|| for every user row, with
        e = entry_bound (default norm_bound), so an error confined to one
        band tile, antenna block or user block fails;
      - per vector: ||dGS[b, :]|| <= e ||gS[b, :]|| for every right-hand
        side b (GS = mu_b, a solve output like x);
      - zero off the band (GH is written only on VR entries).
    Returns the measured ratios."""
    gH, gS, gxi = ref
    e = norm_bound if entry_bound is None else entry_bound
    dH = np.where(mask, g["GH"] - gH, 0)
    r = {
        "gh_norm": np.linalg.norm(dH) / np.linalg.norm(gH[mask]),
        "gs_norm": np.linalg.norm(g["GS"] - gS) / np.linalg.norm(gS),
        "gxi": abs(g["gxi"] - gxi) / abs(gxi),
        "gh_entry": np.abs(dH).max() / np.abs(gH[mask]).max(),
        "gh_row": (np.linalg.norm(dH, axis=1) / np.linalg.norm(gH, axis=1).max()).max(),
        "gs_vec": (np.linalg.norm(g["GS"] - gS, axis=1) / np.maximum(np.linalg.norm(gS, axis=1), 1e-300)).max(),
    }
    print("grad parity %s: %s" % (label, " ".join("%s %.2e" % kv for kv in r.items())), flush=True)
    assert r["gh_norm"] <= norm_bound and r["gs_norm"] <= norm_bound and r["gxi"] <= norm_bound, (label, r)
    assert r["gh_entry"] <= e and r["gh_row"] <= e and r["gs_vec"] <= e, (label, r)
    assert not np.asarray(g["GH"])[~mask].any(), label
    return r
