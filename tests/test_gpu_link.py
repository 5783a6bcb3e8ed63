"""Precoding matrix and link metrics on the GPU (solve on S = I_K, then the
effective channel, beta and per-user spectral efficiency kernels), against
the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _noise(drop):
    """sigma^2 / rho of the rate: the fifth entry of the drop tuple, else xi / K
    (the workloads' regulariser is xi = K sigma^2 / rho)."""
    return drop[4] if len(drop) > 4 else drop[3] / drop[0].shape[0]


def _run(drops, dtype="c64", engine="auto", tol=1e-5):
    """drops: list of (H, vs, vl, xi[, noise]). Solve S = I_K for every drop
    in one plan, then the link metrics; returns per-drop (X, E, rate, beta)."""
    import torch
    from paper_2501_10689_amd import vrk
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    specs, E, R, Bt = [], [], [], []
    for H, vs, vl, xi in (dr[:4] for dr in drops):
        K, Nt = H.shape
        Hd = to_dev(H, tdt)
        S = torch.eye(K, dtype=tdt, device="cuda")
        X = torch.full((K, Nt), float("nan"), dtype=tdt, device="cuda")
        specs.append(vrk.ProblemSpec(Hd, vs, vl, xi, S, X))
        E.append(torch.full((K, K), float("nan"), dtype=tdt, device="cuda"))
        R.append(torch.full((K,), float("nan"), dtype=torch.float64, device="cuda"))
        Bt.append(torch.full((1,), float("nan"), dtype=torch.float64, device="cuda"))
    plan = vrk.Plan(specs, vrk.options(dtype=dtype, engine=engine, tol=tol))
    plan.solve()
    plan.link_metrics(E, R, Bt, [_noise(dr) for dr in drops])
    torch.cuda.synchronize()
    return [(sp.X.cpu().numpy().astype(np.complex128), e.cpu().numpy().astype(np.complex128),
             r.cpu().numpy(), float(b.cpu().numpy()[0])) for sp, e, r, b in zip(specs, E, R, Bt)], plan


def _check(drop, out, e_tol, r_tol, b_tol, nmse_tol, own_tol):
    H, vs, vl, xi = drop[:4]
    nz = _noise(drop)
    X, E, rate, beta = out
    # against the oracle's exact RZF precoder
    Xo = oracle.precoder(H, vs, vl, xi)
    Eo, bo, ro = oracle.link_metrics(H, vs, vl, nz, Xo)
    assert np.max(np.abs(E - Eo)) <= e_tol
    assert np.max(np.abs(rate - ro)) <= r_tol
    assert abs(beta - bo) <= b_tol * bo
    assert oracle.nmse(bo * Xo, beta * X) <= nmse_tol
    # the link kernels alone: the oracle's metrics of the GPU's own precoder
    Eg, bg, rg = oracle.link_metrics(H, vs, vl, nz, X)
    assert np.max(np.abs(E - Eg)) <= own_tol
    assert np.max(np.abs(rate - rg)) <= own_tol
    assert abs(beta - bg) <= 1e-12 * bg


def test_link_metrics_c64_mfma_one_drop():
    d = synth.make_workload("many_rhs", nrhs=1, nt=512, k=48)[0]
    drop = (d.H, d.vr_start, d.vr_len, d.xi)
    out, plan = _run([drop], engine="mfma")
    assert plan.query(0, 5)[0] == 2
    _check(drop, out[0], e_tol=1e-4, r_tol=2e-4, b_tol=5e-5, nmse_tol=1e-4, own_tol=2e-5)


def test_link_metrics_uneven_batch_with_empty_vr():
    # drops of different K and Nt in one plan; one user without any visible
    # antenna (its row of E is zero and so is its rate)
    ds = synth.make_workload("uneven", drops=6, nrhs=1, seed=7)
    drops = []
    for j, d in enumerate(ds):
        H, vs, vl = d.H.copy(), d.vr_start.copy(), d.vr_len.copy()
        if j == 2:
            vl[3] = 0
            H[3] = 0
        drops.append((H, vs, vl, d.xi))
    out, _ = _run(drops, engine="mfma")
    for drop, o in zip(drops, out):
        _check(drop, o, e_tol=1e-4, r_tol=2e-4, b_tol=5e-5, nmse_tol=1e-4, own_tol=2e-5)
    assert np.all(out[2][1][3] == 0) and out[2][2][3] == 0.0


def test_link_metrics_c128_vector_engine():
    d = synth.make_workload("plain", nrhs=1)[0]
    drop = (d.H, d.vr_start, d.vr_len, d.xi)
    out, plan = _run([drop], dtype="c128", tol=1e-10)
    _check(drop, out[0], e_tol=1e-8, r_tol=1e-8, b_tol=1e-8, nmse_tol=1e-8, own_tol=1e-12)


def test_link_metrics_single_user_c64():
    # K = 1 (vector engine): with xi = sigma^2 / rho the rate is
    # log2(1 + |h|^2 / xi); with another noise level n it is log2(1 + beta^2
    # |E|^2 / n), beta^2 |E|^2 = |h|^2 for a single user
    rng = np.random.default_rng(3)
    H = np.zeros((1, 64), dtype=np.complex128)
    H[0, 10:40] = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    h2 = float(np.sum(np.abs(H) ** 2))
    for noise in (0.5, 0.07):
        drop = (H, np.array([10], np.int32), np.array([30], np.int32), 0.5, noise)
        out, _ = _run([drop])
        assert abs(out[0][2][0] - np.log2(1 + h2 / noise)) <= 1e-4


def test_link_metrics_rejects_other_right_hand_sides():
    import torch
    from paper_2501_10689_amd import vrk
    d = synth.make_workload("many_rhs", nrhs=20, nt=256, k=16)[0]
    Hd = to_dev(d.H, torch.complex64)
    S = to_dev(d.S, torch.complex64)
    X = torch.empty((20, 256), dtype=torch.complex64, device="cuda")
    plan = vrk.Plan([vrk.ProblemSpec(Hd, d.vr_start, d.vr_len, d.xi, S, X)], vrk.options())
    plan.solve()
    E = torch.empty((16, 16), dtype=torch.complex64, device="cuda")
    r = torch.empty(16, dtype=torch.float64, device="cuda")
    b = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(vrk.VrkError):
        plan.link_metrics([E], [r], [b], 0.1)
