"""The seeded input generators: shapes, the structural zeros the library's
contract relies on, and reproducibility (CPU)."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def _check_masked(d):
    U = oracle.mask_indicator(d.vr_mask, d.nt, d.n_sub).astype(bool)
    assert np.all(d.H[~U] == 0)                        # h = hbar * u: hidden antennas are zero
    vs, vl = synth.mask_hulls(d.vr_mask, d.nt, d.n_sub)
    assert np.array_equal(vs, d.vr_start) and np.array_equal(vl, d.vr_len)
    for k in range(d.k):                               # nothing outside the hull either
        assert not d.H[k, :d.vr_start[k]].any() and not d.H[k, d.vr_start[k] + d.vr_len[k]:].any()


def test_interval_workloads_are_zero_outside_the_vrs():
    for name in ("plain", "many_rhs", "uneven", "adjoint", "large"):
        for d in synth.make_workload(name, drops=2, nrhs=3, nt=256 if name != "uneven" else None,
                                     k=16 if name != "uneven" else None):
            for k in range(d.k):
                a, b = d.vr_start[k], d.vr_start[k] + d.vr_len[k]
                assert 0 <= a <= b <= d.nt
                assert not d.H[k, :a].any() and not d.H[k, b:].any()
            assert d.S.shape == (3, d.k) and d.xi > 0


def test_subarray_and_paper_drops():
    for d in synth.make_workload("subarray", drops=3, nrhs=4):
        assert (d.nt, d.k, d.n_sub) == (2000, 30, 20) and d.xi == 30.0
        _check_masked(d)
    for d in synth.make_workload("paper", drops=3):
        assert (d.nt, d.k, d.n_sub) == (2000, 30, 20) and d.xi == 1.0 and d.S.shape == (0, 30)
        _check_masked(d)
        n = np.linalg.norm(d.H, axis=1)
        assert np.allclose(n[n > 0], 1.0, rtol=0, atol=1e-12)   # power control: unit-norm rows
    # visibility frequency near p over many draws
    masks = np.concatenate([d.vr_mask for d in synth.make_workload("subarray", drops=40, nrhs=1)])
    frac = np.mean([bin(int(m)).count("1") for m in masks]) / 20
    assert abs(frac - 0.35) < 0.03


def test_multipath_channel_matches_its_definition():
    # one user, one path, all subarrays visible: h_n = g exp(-j 2 pi (d_n - d_0) / lambda) / sqrt(L),
    # so |h| is flat across the array and the phase at the centre antenna is arg g
    rng = np.random.default_rng(1)
    d = synth.make_multipath_drop(rng, nt=64, k=1, n_sub=1, p_vis=1.0, n_paths=1)
    h = d.H[0]
    assert np.allclose(np.abs(h), np.abs(h[0]), rtol=1e-12)
    rng = np.random.default_rng(1)
    r = rng.uniform(1.0, 50.0, size=1)
    th = np.deg2rad(rng.uniform(30.0, 150.0, size=1))
    g = (rng.standard_normal(1) + 1j * rng.standard_normal(1)) * np.sqrt(0.5)
    lam = synth.channels.C_LIGHT / 100e9
    pos = (np.arange(64) - 31.5) * lam / 2
    dn = np.sqrt(r[0] ** 2 + pos ** 2 - 2 * pos * r[0] * np.cos(th[0]))
    want = g[0] * np.exp(-2j * np.pi * (dn - r[0]) / lam)
    want /= np.linalg.norm(want)
    assert np.allclose(h, want, rtol=0, atol=1e-12)


def test_generators_are_reproducible():
    a = synth.make_workload("uneven", drops=3, nrhs=2)
    b = synth.make_workload("uneven", drops=3, nrhs=2)
    for x, y in zip(a, b):
        assert np.array_equal(x.H, y.H) and np.array_equal(x.S, y.S) and x.xi == y.xi
    c = synth.make_workload("uneven", drops=3, nrhs=2, seed=9)
    assert not np.array_equal(a[0].H, c[0].H) or a[0].H.shape != c[0].H.shape
