"""Qualitative claims of the simulation section, reproduced with the FP64
oracle on the subarray VR model (CPU; the paper's figure data are absent, so
only the direction of each trend is checked)."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def _cost(d, variant, nb=3, tol=1e-6):
    """Multiplications of the VR-restricted steps (Table I's counting, VR
    sizes = visible antennas): VR-OGRK pays |Gamma_i| for the update of the
    chosen row i plus the residuals of its overlap set X_i; VR-OAHK pays per
    iteration the residual check, the F half-step, the V residual and the V
    aggregation."""
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    L = d.nt // d.n_sub
    g = np.array([bin(int(m)).count("1") * L for m in d.vr_mask])
    X = oracle.overlap_sets(d.H, d.vr_start, d.vr_len, d.xi, **kw)
    F = oracle.mis(d.H, d.vr_start, d.vr_len, d.xi, **kw)
    tot = 0.0
    for b in range(nb):
        o = oracle.solve(d.H, d.vr_start, d.vr_len, d.S[b], d.xi, variant=variant, tol=tol,
                         trace=variant == "vr_ogrk", max_iters=20000, **kw)
        assert o["flags"] & oracle.F_CONVERGED
        if variant == "vr_ogrk":
            tot += sum(g[i] + g[X[i]].sum() for i in o["idx"][1:])
        else:
            tot += o["iters"] * (g.sum() + g[F].sum() + 2 * g[~F].sum())
    return tot / nb, F.sum()


def test_complexity_grows_with_visibility_probability():
    # Fig. 7's claim: a larger p (weaker spatial non-stationarity) raises the
    # complexity of both VR-OGRK and VR-OAHK, and VR-OAHK stays far cheaper;
    # the orthogonal set shrinks as the VR graph densifies
    rows = []
    for p in (0.1, 0.35, 0.9):
        c = []
        for dd in range(2):
            rng = np.random.default_rng([77, dd, int(p * 100)])
            d = synth.make_subarray_drop(rng, nt=400, k=30, nrhs=3, n_sub=20, p_vis=p, snr_db=0.0)
            og, nf = _cost(d, "vr_ogrk")
            oa, _ = _cost(d, "vr_oahk")
            c.append((og, oa, nf))
        rows.append(np.mean(c, axis=0))
    rows = np.array(rows)
    assert np.all(np.diff(rows[:, 0]) > 0) and np.all(np.diff(rows[:, 1]) > 0)
    assert np.all(rows[:, 1] < rows[:, 0] / 2)
    assert np.all(np.diff(rows[:, 2]) < 0)


def _nmse_first_below(d, variant, t_max, level=1e-6):
    """Smallest per-column iteration count T at which the precoding matrix
    from T iterations on every column of S = I_K (Remark 2) is within NMSE
    `level` of the RZF precoder (both normalised by their beta, the NMSE of
    the simulation section)."""
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    Xo = oracle.precoder(d.H, d.vr_start, d.vr_len, d.xi)
    Fo = Xo / np.linalg.norm(Xo)
    Z = []
    for b in range(d.k):
        e = np.zeros(d.k)
        e[b] = 1.0
        o = oracle.solve(d.H, d.vr_start, d.vr_len, e, d.xi, variant=variant, tol=0.0, max_iters=t_max,
                         trace=True, **kw)
        z = o["z"][:, :d.nt]
        Z.append(z if variant == "vr_ogrk" else z[0::2])   # VR-OAHK traces both half-steps
    for t in range(1, t_max + 1):
        X = np.array([z[min(t, len(z) - 1)] for z in Z])
        if oracle.nmse(Fo, X / np.linalg.norm(X)) <= level:
            return t
    return None


def test_iterations_to_nmse_on_the_paper_setup():
    # Fig. 2's setting (Nt 2000, 100 GHz, S 20, p 0.35, K 30, L_k 5, SNR 0 dB):
    # VR-OAHK reaches NMSE 1e-6 on F in a handful of iterations (the paper
    # quotes 5), VR-OGRK needs several times more (27 there; the figure's
    # data are absent, so only the ordering and the scale are checked)
    d = synth.make_multipath_drop(np.random.default_rng([6, 0, 0]))
    t_oahk = _nmse_first_below(d, "vr_oahk", 20)
    t_ogrk = _nmse_first_below(d, "vr_ogrk", 200)
    assert t_oahk is not None and 3 <= t_oahk <= 10
    assert t_ogrk is not None and t_ogrk >= 3 * t_oahk


def test_fig2_ordering_uniform_rk_vs_vr_variants():
    # Fig. 2's ordering on the paper's setting: to reach NMSE 1e-6 on F, the
    # uniform-criterion RK (URK) needs many more iterations than VR-OGRK,
    # which needs many more than VR-OAHK. Rows have unit norm here, so the
    # energy criterion coincides with the uniform one (the second limitation
    # the paper names for energy-based selection)
    d = synth.make_multipath_drop(np.random.default_rng([6, 0, 0]))
    kw = dict(masks=d.vr_mask, n_sub=d.n_sub)
    nrm = oracle.row_norms(d.H, d.vr_start, d.vr_len, d.xi, **kw)
    assert np.ptp(nrm) <= 1e-12 * nrm.max()
    Xo = oracle.precoder(d.H, d.vr_start, d.vr_len, d.xi)
    Fo = Xo / np.linalg.norm(Xo)

    def nmse_after(variant, select, T):
        X = oracle.solve_batch(d.H, d.vr_start, d.vr_len, np.eye(d.k), d.xi, variant=variant, select=select,
                               tol=0.0, max_iters=T, **kw)["X"]
        return oracle.nmse(Fo, X / np.linalg.norm(X))

    t_oahk = _nmse_first_below(d, "vr_oahk", 20)
    t_ogrk = _nmse_first_below(d, "vr_ogrk", 200)
    assert t_ogrk >= 3 * t_oahk
    # URK is still far from NMSE 1e-6 after three times VR-OGRK's count
    assert nmse_after("grk", "uniform", 3 * t_ogrk) > 1e-4
    # ... and gets there eventually (same fixed point)
    assert nmse_after("grk", "uniform", 1600) <= 1e-6
    assert nmse_after("grk", "energy", 1600) <= 1e-6
