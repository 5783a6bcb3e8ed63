"""Differentiation through the library: KaczmarzRZF.backward runs the
adjoint Kaczmarz solve. Checked with FP64 finite differences (torch
gradcheck, Nt 64, K 8) and against the oracle's closed-form gradient on the
adjoint workload shape."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import random_problem

pytestmark = pytest.mark.gpu


def test_gradcheck_fp64_finite_differences():
    import torch
    from paper_2501_10689_amd.autograd import rzf_precode
    rng = np.random.default_rng(3)
    H, vs, vl, xi = random_problem(rng, 64, 8)
    S = (rng.standard_normal((3, 8)) + 1j * rng.standard_normal((3, 8))) / np.sqrt(2)
    Ht = torch.tensor(H, device="cuda", requires_grad=True)
    St = torch.tensor(S, device="cuda", requires_grad=True)
    xit = torch.tensor(xi, dtype=torch.float64, device="cuda", requires_grad=True)

    def f(Hh, Ss, xx):
        X = rzf_precode(Hh, Ss, xx, vs, vl, variant="vr_oahk", engine="vector", tol=1e-14)
        R = X @ Hh.T.contiguous() - Ss
        return (R.abs().pow(2).sum() + 0.1 * X.abs().pow(2).sum()) / 3

    assert torch.autograd.gradcheck(f, (Ht, St, xit), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)


@pytest.mark.parametrize("variant", ["vr_oahk", "ahk", "grk"])
def test_autograd_matches_closed_form_adjoint_workload(variant):
    """Nt 1024, K 64, 64 QPSK vectors, SNR 10 dB (one drop of the adjoint
    workload), loss mean ||H x - s||^2 + 0.1 ||x||^2, complex64."""
    import torch
    from paper_2501_10689_amd.autograd import rzf_precode
    d = synth.make_workload("adjoint", drops=1)[0]
    Ht = torch.tensor(d.H, dtype=torch.complex64, device="cuda", requires_grad=True)
    St = torch.tensor(d.S, dtype=torch.complex64, device="cuda", requires_grad=True)
    xit = torch.tensor(d.xi, dtype=torch.float64, device="cuda", requires_grad=True)
    mask = torch.tensor(np.abs(d.H) > 0, device="cuda")
    Hm = Ht * mask   # the channel equation's VR mask: off-band entries are structural zeros
    X = rzf_precode(Hm, St, xit, d.vr_start, d.vr_len, variant=variant, tol=1e-6)
    R = X @ Hm.T.contiguous() - St
    L = (R.abs().pow(2).sum() + 0.1 * X.abs().pow(2).sum()) / d.nrhs
    L.backward()
    Xr, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    Rr = Xr @ d.H.T - d.S
    G = 2.0 * (Rr @ d.H.conj() + 0.1 * Xr) / d.nrhs
    gH, gS, gxi = oracle.rzf_grad(d.H, d.vr_start, d.vr_len, d.S, d.xi, G)
    m = np.abs(d.H) > 0
    gH = gH + 2.0 * (Rr.T @ Xr.conj()) / d.nrhs * m
    gS = gS - 2.0 * Rr / d.nrhs
    eH = np.linalg.norm((Ht.grad.cpu().numpy() - gH)[m]) / np.linalg.norm(gH[m])
    eS = np.linalg.norm(St.grad.cpu().numpy() - gS) / np.linalg.norm(gS)
    exi = abs(float(xit.grad) - gxi) / abs(gxi)
    print(variant, "rel err dH %.2e dS %.2e dxi %.2e" % (eH, eS, exi))
    assert eH <= 1e-4 and eS <= 1e-4 and exi <= 1e-4
    assert not Ht.grad.cpu().numpy()[~m].any()
    # entry by entry (relative to the largest band entry), per user row and
    # per right-hand side
    dH = np.where(m, Ht.grad.cpu().numpy() - gH, 0)
    dS = St.grad.cpu().numpy() - gS
    assert np.abs(dH).max() <= 5e-4 * np.abs(gH[m]).max()
    assert np.linalg.norm(dH, axis=1).max() <= 5e-4 * np.linalg.norm(gH, axis=1).max()
    assert (np.linalg.norm(dS, axis=1) / np.linalg.norm(gS, axis=1)).max() <= 5e-4
