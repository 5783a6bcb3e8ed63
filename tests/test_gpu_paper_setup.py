"""The simulation setting of the paper on the GPU (Nt 2000 at 100 GHz, S 20
subarrays visible w.p. 0.35, K 30 users, L_k 5 near-field paths, SNR 0 dB):
precoding matrices from a fixed number of iterations per column of
S = I_K (the fixed-T runs behind Fig. 2 and Fig. 3), against the FP64
oracle's iterates after the same number of steps."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel_err_rows, run_plan

pytestmark = pytest.mark.gpu


def _drop(seed=0, snr_db=0.0):
    return synth.make_multipath_drop(np.random.default_rng([6, seed, 0]), snr_db=snr_db)


def _oracle_X(d, variant, T):
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    rows = []
    for b in range(d.k):
        e = np.zeros(d.k)
        e[b] = 1.0
        rows.append(oracle.solve(d.H, d.vr_start, d.vr_len, e, d.xi, variant=variant, tol=0.0, max_iters=T,
                                 rhs=b, **kw)["x"])
    return np.array(rows)


def _gpu_X(d, variant, T, dtype, engine):
    res, _ = run_plan([(d.H, d.vr_start, d.vr_len, np.eye(d.k), d.xi, d.vr_mask, d.n_sub)], variant=variant,
                      dtype=dtype, engine=engine, tol=0.0, max_iters=T)
    r = res[0]
    assert np.all(r["flags"] == oracle.F_MAXITER) and np.all(r["iters"] == T)
    return r["X"]


@pytest.mark.parametrize("variant,T", [("vr_oahk", 1), ("vr_oahk", 4), ("vr_oahk", 7),
                                       ("vr_ogrk", 5), ("vr_ogrk", 40)])
def test_fixed_iteration_precoder_c128_equals_oracle_iterate(variant, T):
    d = _drop()
    Xg = _gpu_X(d, variant, T, "c128", "vector")
    Xo = _oracle_X(d, variant, T)
    assert rel_err_rows(Xg, Xo).max() <= 1e-9


def test_nmse_curve_c64_mfma_follows_oracle():
    # VR-OAHK on the matrix cores: NMSE of beta F after T iterations per
    # column, T = 1..5 (6e-2 down to ~1e-5), against the oracle's curve
    d = _drop(1)
    Xr = oracle.precoder(d.H, d.vr_start, d.vr_len, d.xi)
    Fr = Xr / np.linalg.norm(Xr)
    for T in range(1, 6):
        Xg = _gpu_X(d, "vr_oahk", T, "c64", "mfma")
        Xo = _oracle_X(d, "vr_oahk", T)
        ng = oracle.nmse(Fr, Xg / np.linalg.norm(Xg))
        no = oracle.nmse(Fr, Xo / np.linalg.norm(Xo))
        assert abs(ng - no) <= 0.02 * no + 2e-7, (T, ng, no)


def test_rates_after_fifteen_iterations():
    # Fig. 3's fixed budget T = 15: per-user spectral efficiency of the
    # precoder after 15 iterations, from the link-metric kernels, against the
    # oracle's metrics of its own 15-step iterate; VR-OAHK is then at the RZF
    import torch
    from paper_2501_10689_amd import vrk
    d = _drop(2, snr_db=10.0)
    Hd = torch.tensor(d.H, dtype=torch.complex64, device="cuda")
    S = torch.eye(d.k, dtype=torch.complex64, device="cuda")
    for variant in ("vr_oahk", "vr_ogrk"):
        X = torch.zeros((d.k, d.nt), dtype=torch.complex64, device="cuda")
        plan = vrk.Plan([vrk.ProblemSpec(Hd, d.vr_start, d.vr_len, d.xi, S, X, vr_mask=d.vr_mask,
                                         n_sub=d.n_sub)],
                        vrk.options(variant=variant, tol=0.0, max_iters=15, engine="mfma"))
        plan.solve()
        E = torch.zeros((d.k, d.k), dtype=torch.complex64, device="cuda")
        R = torch.zeros(d.k, dtype=torch.float64, device="cuda")
        B = torch.zeros(1, dtype=torch.float64, device="cuda")
        plan.link_metrics([E], [R], [B], d.xi)   # xi = sigma^2 / rho on this setting
        torch.cuda.synchronize()
        Xo = _oracle_X(d, variant, 15)
        _, bo, ro = oracle.link_metrics(d.H, d.vr_start, d.vr_len, d.xi, Xo)
        assert np.max(np.abs(R.cpu().numpy() - ro)) <= 2e-4 * max(1.0, ro.max())
        assert abs(float(B.cpu()[0]) - bo) <= 1e-4 * bo
        if variant == "vr_oahk":
            _, _, rr = oracle.link_metrics(d.H, d.vr_start, d.vr_len, d.xi,
                                           oracle.precoder(d.H, d.vr_start, d.vr_len, d.xi))
            assert abs(R.cpu().numpy().sum() - rr.sum()) <= 1e-3 * rr.sum()


def test_precoder_helper_on_the_paper_setting():
    # vrk.precoder with the subarray masks: converged precoding matrix, E,
    # beta and rates against the FP64 RZF and its link metrics
    import torch
    from paper_2501_10689_amd import vrk
    d = _drop(3, snr_db=10.0)
    Hd = torch.tensor(d.H, dtype=torch.complex64, device="cuda")
    X, E, rate, beta = vrk.precoder(Hd, d.vr_start, d.vr_len, d.xi, d.xi, tol=1e-6, vr_mask=d.vr_mask,
                                    n_sub=d.n_sub)
    torch.cuda.synchronize()
    Xr = oracle.precoder(d.H, d.vr_start, d.vr_len, d.xi)
    Er, br, rr = oracle.link_metrics(d.H, d.vr_start, d.vr_len, d.xi, Xr)
    Xg = X.cpu().numpy().astype(np.complex128)
    assert oracle.nmse(br * Xr, beta * Xg) <= 1e-4
    assert np.max(np.abs(E.cpu().numpy() - Er)) <= 1e-4
    assert np.max(np.abs(rate.cpu().numpy() - rr)) <= 2e-4 * max(1.0, rr.max())
    assert abs(beta - br) <= 1e-4 * br
