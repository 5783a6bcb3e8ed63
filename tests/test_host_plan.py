"""Host-side tests of libvrk.so (no GPU needed): the C ABI loads and exports
every function include/vrk.h declares, argument validation, and the VR
plan (overlap sets, orthogonal set F, colour classes) against the oracle
and brute force."""
from __future__ import annotations

import inspect
import itertools
import os
import re

import numpy as np
import pytest

import oracle
from paper_2501_10689_amd import vrk
from tests.helpers import random_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "vrk.h")).read()
    names = set(re.findall(r"^(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vrk_[a-z_0-9]+)\(", hdr, re.M))
    assert {"vrk_plan_create", "vrk_plan_bind", "vrk_solve", "vrk_solve_adjoint"} <= names
    L = vrk.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


def test_build_entry_resolves_its_compile_steps():
    import __graft_entry__
    steps = __graft_entry__._builders()
    assert len(steps) == 2 and all(inspect.isfunction(f) for f in steps)


def test_plan_matches_oracle_structure():
    rng = np.random.default_rng(0)
    for trial in range(30):
        nt, k = int(rng.integers(16, 200)), int(rng.integers(1, 40))
        H, vs, vl, xi = random_problem(rng, nt, k, lo=0, hi=max(1, nt // 2))
        hp = vrk.host_plan(nt, k, vs, vl, xi, engine="vector")
        f = np.zeros(k, dtype=bool)
        f[hp.query(vrk.Q_FSET)] = True
        assert np.array_equal(f, oracle.mis(H, vs, vl, xi))
        xoff, xidx = hp.query(vrk.Q_XOFF), hp.query(vrk.Q_XIDX)
        want = oracle.overlap_sets(H, vs, vl, xi)
        for i in range(k):
            assert np.array_equal(xidx[xoff[i]:xoff[i + 1]], want[i])
        perm = hp.query(vrk.Q_PERM)
        assert sorted(perm.tolist()) == list(range(k))
        keys = [(vs[u], vs[u] + vl[u], u) for u in perm]
        assert keys == sorted(keys)


def _max_clique(vs, vl):
    ev = []
    for s, l in zip(vs, vl):
        if l > 0:
            ev += [(s, 1), (s + l, -1)]
    ev.sort(key=lambda e: (e[0], e[1]))   # ends before starts at the same antenna
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_colour_classes_are_disjoint_and_optimal():
    rng = np.random.default_rng(1)
    for trial in range(40):
        nt, k = 120, int(rng.integers(1, 30))
        H, vs, vl, xi = random_problem(rng, nt, k, lo=0, hi=60)
        col = vrk.host_plan(nt, k, vs, vl, xi, engine="vector").query(vrk.Q_COLOUR)
        for a, b in itertools.combinations(range(k), 2):
            if col[a] == col[b]:
                assert max(vs[a], vs[b]) >= min(vs[a] + vl[a], vs[b] + vl[b])
        assert col.max() + 1 == max(1, _max_clique(vs, vl))


@pytest.mark.parametrize("bad", ["xi0", "xinan", "vrout", "vrneg", "ldh", "tol", "iters", "variant"])
def test_validation_errors(bad):
    vs = np.array([0, 10], dtype=np.int32)
    vl = np.array([8, 6], dtype=np.int32)
    kw = dict(engine="vector")
    nt, k, xi = 32, 2, 1.0
    if bad == "xi0":
        xi = 0.0
    elif bad == "xinan":
        xi = float("nan")
    elif bad == "vrout":
        vl[1] = 23
    elif bad == "vrneg":
        vs[0] = -1
    elif bad == "tol":
        kw["tol"] = -1.0
    elif bad == "iters":
        kw["max_iters"] = 0
    elif bad == "variant":
        kw["variant"] = 7
    if bad == "ldh":
        p = vrk.Problem()
        p.nt, p.k, p.xi, p.H, p.ldh = nt, k, xi, 256, nt - 1
        p.vr_start, p.vr_len = vs.ctypes.data, vl.ctypes.data
        import ctypes as C
        ws, h = C.c_size_t(), C.c_void_p()
        o = vrk.options(**kw)
        st = vrk.lib().vrk_plan_create(C.byref(p), 1, C.byref(o), C.byref(ws), C.byref(h))
        assert st == 1
        return
    with pytest.raises(vrk.VrkError) as e:
        vrk.host_plan(nt, k, vs, vl, xi, **kw)
    assert e.value.status == 1


def test_solve_before_bind_is_a_state_error():
    import ctypes as C
    vs = np.array([0], dtype=np.int32)
    vl = np.array([4], dtype=np.int32)
    p = vrk.Problem()
    p.nt, p.k, p.xi, p.H, p.ldh = 8, 1, 1.0, 256, 8
    p.vr_start, p.vr_len = vs.ctypes.data, vl.ctypes.data
    o = vrk.options(engine="vector")
    ws, h = C.c_size_t(), C.c_void_p()
    assert vrk.lib().vrk_plan_create(C.byref(p), 1, C.byref(o), C.byref(ws), C.byref(h)) == 0
    assert vrk.lib().vrk_solve(h, None, None, None, None) == 5
    assert vrk.lib().vrk_solve_adjoint(h, None, None, None, None) == 5
    assert vrk.lib().vrk_plan_bind(h, None, 0, None) == 3
    vrk.lib().vrk_plan_destroy(h)


# ---------------------------------------------------------------------------
# Subarray VR model: overlap and F from the masks, bit-exact against the
# oracle; colour classes on the hulls; argument checks
# ---------------------------------------------------------------------------

def _bernoulli_masks(rng, k, n_sub, p):
    return np.array([sum(1 << s for s in range(n_sub) if rng.random() < p) for _ in range(k)],
                    dtype=np.uint64)


@pytest.mark.parametrize("engine", ["vector", "mfma"])
def test_masked_plan_matches_oracle_structure(engine):
    import synth
    rng = np.random.default_rng(5)
    for trial in range(40):
        n_sub = int(rng.choice([4, 8, 20, 64]))
        nt = n_sub * int(rng.integers(1, 6))
        k = int(rng.integers(1, 60))
        p = float(rng.uniform(0.05, 0.6))
        masks = _bernoulli_masks(rng, k, n_sub, p)
        if trial % 5 == 0:
            masks[0] = 0                      # a user that sees nothing
        vs, vl = synth.mask_hulls(masks, nt, n_sub)
        H = np.zeros((k, nt), complex)
        hp = vrk.host_plan(nt, k, vs, vl, 1.0, nrhs=16 if engine == "mfma" else 0, vr_mask=masks,
                           n_sub=n_sub, engine=engine)
        f = np.zeros(k, dtype=bool)
        f[hp.query(vrk.Q_FSET)] = True
        assert np.array_equal(f, oracle.mis(H, vs, vl, 1.0, masks=masks, n_sub=n_sub)), trial
        xoff, xidx = hp.query(vrk.Q_XOFF), hp.query(vrk.Q_XIDX)
        want = oracle.overlap_sets(H, vs, vl, 1.0, masks=masks, n_sub=n_sub)
        for i in range(k):
            assert np.array_equal(xidx[xoff[i]:xoff[i + 1]], want[i])
        # colour classes: a greedy colouring of the mask graph in VR-start
        # order (the colour schedule writes only visible antennas)
        col = hp.query(vrk.Q_COLOUR)
        adj = oracle.mask_graph(masks)
        assert not np.any(adj & (col[:, None] == col[None, :]))
        want = np.zeros(k, np.int64)
        seen = []
        for u in hp.query(vrk.Q_PERM):
            used = {want[v] for v in seen if adj[u, v]}
            want[u] = min(c for c in range(k + 1) if c not in used)
            seen.append(u)
        assert np.array_equal(col, want)
        assert col.max() <= adj.sum(axis=1).max()


def test_masked_gram_pattern_is_smaller_than_the_hulls():
    # users u < 32 see subarrays u and u + 32: every hull overlaps every
    # other, no two masks do; the other 32 users see nothing. Under the
    # masks F is everyone and the Gram pattern keeps only the chunks on the
    # diagonal
    import synth
    nt, n_sub, k = 128, 64, 64
    masks = np.array([(1 << u) | (1 << (u + 32)) for u in range(32)] + [0] * 32, dtype=np.uint64)
    vs, vl = synth.mask_hulls(masks, nt, n_sub)
    hp_m = vrk.host_plan(nt, k, vs, vl, 1.0, nrhs=16, vr_mask=masks, n_sub=n_sub, engine="mfma")
    hp_h = vrk.host_plan(nt, k, vs, vl, 1.0, nrhs=16, engine="mfma")
    assert len(hp_m.query(vrk.Q_FSET)) == k
    assert len(hp_h.query(vrk.Q_FSET)) == 33
    assert hp_m.query(vrk.Q_TILES)[3] == 16
    assert hp_h.query(vrk.Q_TILES)[3] == 24


@pytest.mark.parametrize("bad", ["hull", "bits", "nsub0", "nsubdiv", "nsub65"])
def test_masked_validation_errors(bad):
    import synth
    nt, n_sub, k = 40, 8, 3
    masks = np.array([0b00100101, 0b00011000, 0], dtype=np.uint64)
    vs, vl = synth.mask_hulls(masks, nt, n_sub)
    if bad == "hull":
        vl[0] -= 5
    elif bad == "bits":
        masks[1] |= np.uint64(1 << 9)
    elif bad == "nsub0":
        n_sub = 0
    elif bad == "nsubdiv":
        n_sub = 7
    elif bad == "nsub65":
        n_sub = 65
    with pytest.raises(vrk.VrkError) as e:
        vrk.host_plan(nt, k, vs, vl, 1.0, vr_mask=masks, n_sub=n_sub, engine="vector")
    assert e.value.status == 1


def test_adjoint_tile_shape_choice():
    # MFMA plans with adjoint buffers and at most 64 users run the adjoint
    # solve on 8-wave tiles when the tile size is left to the plan
    vs = np.zeros(48, np.int32)
    vl = np.full(48, 100, np.int32)
    q = vrk.host_plan(256, 48, vs, vl, nrhs=32, adjoint=True, engine="mfma").query(vrk.Q_ENGINE)
    assert q[2] == 16 and q[9] == 8
    q = vrk.host_plan(256, 48, vs, vl, nrhs=32, adjoint=True, engine="mfma", tile_waves=16).query(vrk.Q_ENGINE)
    assert q[2] == 16 and q[9] == 16
    q = vrk.host_plan(256, 48, vs, vl, nrhs=32, engine="mfma").query(vrk.Q_ENGINE)
    assert q[9] == 16                      # no adjoint buffers: one shape
    vs2 = np.zeros(100, np.int32)
    vl2 = np.full(100, 100, np.int32)
    q = vrk.host_plan(256, 100, vs2, vl2, nrhs=32, adjoint=True, engine="mfma").query(vrk.Q_ENGINE)
    assert q[9] == q[2] == 16


def test_binding_rejects_host_tensors_before_the_library():
    """The Python binding checks what raw pointers cannot show: a host
    (CPU) tensor for a device buffer is a ValueError, raised before any
    call into libvrk.so."""
    import torch
    H = torch.zeros((4, 32), dtype=torch.complex64)
    S = torch.zeros((3, 4), dtype=torch.complex64)
    X = torch.zeros((3, 32), dtype=torch.complex64)
    sp = vrk.ProblemSpec(H, np.zeros(4, np.int32), np.full(4, 8, np.int32), 1.0, S, X)
    with pytest.raises(ValueError, match="device"):
        vrk.Plan([sp], vrk.options())


def test_wave_owned_tile_choice():
    """Aggregated sweeps get wave-owned tiles (two 16-user blocks per wave,
    so the waves per tile follow K) when tiles x waves per tile reach 4096;
    fewer tiles, the greedy sweeps, an explicit block-tile request or tile
    size keep block tiles; unsupported requests are refused."""
    rng = np.random.default_rng(3)
    H, vs, vl, xi = random_problem(rng, 1024, 64)
    big = vrk.host_plan(1024, 64, vs, vl, nrhs=2048 * 16, variant="vr_oahk")
    assert tuple(big.query(vrk.Q_ENGINE)[10:12]) == (2, 2)
    for kw in (dict(nrhs=2047 * 16), dict(nrhs=2048 * 16, variant="grk"), dict(nrhs=2048 * 16, wave_tiles=-1),
               dict(nrhs=2048 * 16, tile_waves=16)):
        kw.setdefault("variant", "vr_oahk")
        assert vrk.host_plan(1024, 64, vs, vl, **kw).query(vrk.Q_ENGINE)[10] == 0, kw
    H2, vs2, vl2, _ = random_problem(rng, 4096, 256, lo=256, hi=1024)
    p = vrk.host_plan(4096, 256, vs2, vl2, nrhs=512 * 16, variant="ahk")
    assert tuple(p.query(vrk.Q_ENGINE)[10:12]) == (8, 2)
    H3, vs3, vl3, _ = random_problem(rng, 512, 30)
    assert tuple(vrk.host_plan(512, 30, vs3, vl3, nrhs=4096 * 16, variant="vr_oahk")
                 .query(vrk.Q_ENGINE)[10:12]) == (1, 2)
    assert vrk.host_plan(512, 30, vs3, vl3, nrhs=4095 * 16, variant="vr_oahk").query(vrk.Q_ENGINE)[10] == 0
    assert tuple(vrk.host_plan(4096, 256, vs2, vl2, nrhs=64, variant="ahk", wave_tiles=8)
                 .query(vrk.Q_ENGINE)[10:12]) == (8, 2)
    with pytest.raises(vrk.VrkError):
        vrk.host_plan(4096, 256, vs2, vl2, nrhs=64, variant="ahk", wave_tiles=2)   # 16 blocks on 2 waves
    with pytest.raises(vrk.VrkError):
        vrk.host_plan(1024, 64, vs, vl, nrhs=64, variant="grk", wave_tiles=1)


def test_small_channel_vector_form_choice():
    """The vector engine takes its small-channel form (one wave per 64-antenna
    slot, at most four, per right-hand side) when nt <= 1024, k <= 64, the
    VRs are intervals and the channel, zero-padded to 16-row blocks, fits
    128 KiB of LDS, and
    the general four-wave form otherwise; tile_waves 1 or 4 forces the form
    (1 refused where it does not fit) and selects the vector engine under
    AUTO. Q_ENGINE reports 1 and 4 for the two forms."""
    rng = np.random.default_rng(4)
    _, vs, vl, _ = random_problem(rng, 256, 16)
    small = vrk.host_plan(256, 16, vs, vl, nrhs=1, dtype="c128", engine="vector")
    assert small.query(vrk.Q_ENGINE)[2] == 1
    assert vrk.host_plan(256, 16, vs, vl, nrhs=1, dtype="c128", engine="vector",
                         tile_waves=4).query(vrk.Q_ENGINE)[2] == 4
    q = vrk.host_plan(256, 16, vs, vl, nrhs=64, dtype="c64", tile_waves=1).query(vrk.Q_ENGINE)
    assert (q[0], q[2]) == (vrk.ENGINES["vector"], 1)
    # 64 users x 1024 antennas: 1 MiB in complex128
    _, vs1, vl1, _ = random_problem(rng, 1024, 64)
    assert vrk.host_plan(1024, 64, vs1, vl1, nrhs=1, dtype="c128", engine="vector").query(vrk.Q_ENGINE)[2] == 4
    with pytest.raises(vrk.VrkError):
        vrk.host_plan(1024, 64, vs1, vl1, nrhs=1, dtype="c128", engine="vector", tile_waves=1)
    # rows pad to 16: 16 x 1024 complex64 and 64 x 128 complex128 (128 KiB)
    # fit, 16 x 1024 complex128 and 48 x 256 complex128 do not
    _, vs2, vl2, _ = random_problem(rng, 1000, 8)
    assert vrk.host_plan(1000, 8, vs2, vl2, nrhs=1, dtype="c64", engine="vector").query(vrk.Q_ENGINE)[2] == 1
    assert vrk.host_plan(1000, 8, vs2, vl2, nrhs=1, dtype="c128", engine="vector").query(vrk.Q_ENGINE)[2] == 4
    _, vs3, vl3, _ = random_problem(rng, 100, 64)
    assert vrk.host_plan(100, 64, vs3, vl3, nrhs=1, dtype="c128", engine="vector").query(vrk.Q_ENGINE)[2] == 1
    _, vs4, vl4, _ = random_problem(rng, 256, 33)
    assert vrk.host_plan(256, 33, vs4, vl4, nrhs=1, dtype="c128", engine="vector").query(vrk.Q_ENGINE)[2] == 4
    assert vrk.host_plan(256, 33, vs4, vl4, nrhs=1, dtype="c64", engine="vector").query(vrk.Q_ENGINE)[2] == 1
    _, vs5, vl5, _ = random_problem(rng, 2048, 16)
    assert vrk.host_plan(2048, 16, vs5, vl5, nrhs=1, engine="vector").query(vrk.Q_ENGINE)[2] == 4
    _, vs6, vl6, _ = random_problem(rng, 256, 65)
    assert vrk.host_plan(256, 65, vs6, vl6, nrhs=1, engine="vector").query(vrk.Q_ENGINE)[2] == 4
    with pytest.raises(vrk.VrkError):
        vrk.host_plan(256, 16, vs, vl, nrhs=1, tile_waves=2)
