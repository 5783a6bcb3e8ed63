"""Synthetic near-field channels with contiguous visibility regions (VRs).

Channel model (system model, Sec. II-A/B of the paper, simplified to one
line-of-sight spherical-wave path plus optional Rayleigh scattering on the
visible antennas):

* ULA of ``nt`` antennas at half-wavelength spacing ``d = lambda/2``, antenna
  ``n`` at ``((n - (nt-1)/2) d, 0)``.
* User ``k`` at range ``r_k`` and angle ``theta_k`` measured from broadside,
  i.e. at ``(r sin(theta), r cos(theta))``; its distance to antenna ``n`` is
  ``r_kn = sqrt(r^2 + delta_n^2 - 2 r delta_n sin(theta))`` (law of cosines).
* ``H[k, n] = exp(-j 2 pi r_kn / lambda) / r_kn (+ CN(0, nlos_var))`` for
  ``n`` in the VR ``[start_k, start_k + len_k)`` and exactly zero elsewhere
  (the VR mask of the channel equation with its indicator vector).

Row ``k`` of ``H`` (shape ``K x Nt``) is what user ``k`` sees, so the
received signal is ``y_k = sum_n H[k, n] x[n]``; the paper's channel matrix
is the conjugate transpose of this array.

Randomness: ``numpy.random.Generator(PCG64(SeedSequence([cfg, seed, drop])))``,
drawing per drop, in order: (per-drop shape/SNR draws, if any), ranges,
angles, VR lengths, VR starts, NLoS band entries (user by user), symbols.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299_792_458.0


@dataclasses.dataclass
class Drop:
    """One channel drop with its symbol batch. Arrays are complex128."""

    H: np.ndarray          # (K, Nt) complex128, zero outside each VR
    vr_start: np.ndarray   # (K,) int32
    vr_len: np.ndarray     # (K,) int32
    S: np.ndarray          # (B, K) complex128, one symbol vector per row
    xi: float              # regulariser K / SNR_linear
    snr_db: float
    vr_mask: np.ndarray | None = None   # (K,) uint64 visible subarrays, subarray model only
    n_sub: int = 0                      # subarrays S of the subarray model

    @property
    def nt(self) -> int:
        return int(self.H.shape[1])

    @property
    def k(self) -> int:
        return int(self.H.shape[0])

    @property
    def nrhs(self) -> int:
        return int(self.S.shape[0])


def qpsk(rng: np.random.Generator, shape) -> np.ndarray:
    """Unit-energy QPSK symbols (+-1 +-j)/sqrt(2)."""
    b = rng.integers(0, 2, size=tuple(shape) + (2,))
    v = (2.0 * b - 1.0) / math.sqrt(2.0)
    return v[..., 0] + 1j * v[..., 1]


def qam16(rng: np.random.Generator, shape) -> np.ndarray:
    """Unit-energy 16-QAM symbols, levels {+-1, +-3}/sqrt(10) per axis."""
    lv = np.array([-3.0, -1.0, 1.0, 3.0]) / math.sqrt(10.0)
    i = rng.integers(0, 4, size=tuple(shape) + (2,))
    v = lv[i]
    return v[..., 0] + 1j * v[..., 1]


def make_drop(rng: np.random.Generator, *, nt: int, k: int, nrhs: int,
              vr_lo: int, vr_hi: int, snr_db: float, fc: float = 28e9,
              r_lo: float = 5.0, r_hi: float = 50.0, ang_deg: float = 60.0,
              nlos_var: float = 0.0, symbols: str = "qpsk") -> Drop:
    """Draw one drop. VR lengths are integers uniform in [vr_lo, vr_hi]
    (inclusive, clipped to [0, nt]); starts are uniform in [0, nt - len]."""
    lam = C_LIGHT / fc
    d = lam / 2.0
    r = rng.uniform(r_lo, r_hi, size=k)
    th = np.deg2rad(rng.uniform(-ang_deg, ang_deg, size=k))
    lo = max(0, min(vr_lo, nt))
    hi = max(lo, min(vr_hi, nt))
    vlen = rng.integers(lo, hi + 1, size=k).astype(np.int32)
    vstart = np.array([rng.integers(0, nt - L + 1) for L in vlen], dtype=np.int32)
    H = np.zeros((k, nt), dtype=np.complex128)
    delta = (np.arange(nt) - (nt - 1) / 2.0) * d
    for u in range(k):
        a, L = int(vstart[u]), int(vlen[u])
        if L == 0:
            continue
        dn = delta[a:a + L]
        rk = np.sqrt(r[u] ** 2 + dn ** 2 - 2.0 * r[u] * dn * np.sin(th[u]))
        H[u, a:a + L] = np.exp(-2j * np.pi * rk / lam) / rk
    if nlos_var > 0.0:
        sd = math.sqrt(nlos_var / 2.0)
        for u in range(k):
            a, L = int(vstart[u]), int(vlen[u])
            g = rng.standard_normal((L, 2)) * sd
            H[u, a:a + L] += g[:, 0] + 1j * g[:, 1]
    if symbols == "qpsk":
        S = qpsk(rng, (nrhs, k))
    elif symbols == "qam16":
        S = qam16(rng, (nrhs, k))
    else:
        raise ValueError(symbols)
    xi = k / (10.0 ** (snr_db / 10.0))
    return Drop(H=H, vr_start=vstart, vr_len=vlen, S=S, xi=float(xi), snr_db=float(snr_db))


def mask_hulls(masks, nt: int, n_sub: int):
    """Per-user (vr_start, vr_len) of the smallest antenna interval holding
    every visible subarray (0, 0 for a user that sees none)."""
    L = nt // n_sub
    vs = np.zeros(len(masks), dtype=np.int32)
    vl = np.zeros(len(masks), dtype=np.int32)
    for k, m in enumerate(masks):
        bits = [s for s in range(n_sub) if (int(m) >> s) & 1]
        if bits:
            vs[k] = bits[0] * L
            vl[k] = (bits[-1] + 1) * L - vs[k]
    return vs, vl


def make_subarray_drop(rng: np.random.Generator, *, nt: int, k: int, nrhs: int, n_sub: int,
                       p_vis: float, snr_db: float, fc: float = 100e9, r_lo: float = 1.0,
                       r_hi: float = 50.0, ang_deg: float = 60.0, nlos_var: float = 0.1,
                       symbols: str = "qpsk") -> Drop:
    """Draw one drop of the subarray VR model: the array is split into
    ``n_sub`` subarrays of ``nt / n_sub`` antennas and each subarray is
    visible to each user independently with probability ``p_vis``. The
    channel is the spherical-wave LoS path (+ CN(0, nlos_var)) on the
    visible antennas and exactly zero on the hidden ones, so each user's
    interval (the hull of its visible subarrays) may hold zero gaps.
    Draw order: ranges, angles, visibility (user by user, subarray by
    subarray), NLoS entries (user by user over the hull), symbols."""
    if nt % n_sub or not 1 <= n_sub <= 64:
        raise ValueError("nt must be a multiple of n_sub, 1 <= n_sub <= 64")
    lam = C_LIGHT / fc
    d = lam / 2.0
    L = nt // n_sub
    r = rng.uniform(r_lo, r_hi, size=k)
    th = np.deg2rad(rng.uniform(-ang_deg, ang_deg, size=k))
    vis = rng.random((k, n_sub)) < p_vis
    masks = np.array([sum(1 << s for s in range(n_sub) if vis[u, s]) for u in range(k)],
                     dtype=np.uint64)
    vstart, vlen = mask_hulls(masks, nt, n_sub)
    delta = (np.arange(nt) - (nt - 1) / 2.0) * d
    H = np.zeros((k, nt), dtype=np.complex128)
    for u in range(k):
        rk = np.sqrt(r[u] ** 2 + delta ** 2 - 2.0 * r[u] * delta * np.sin(th[u]))
        H[u] = np.exp(-2j * np.pi * rk / lam) / rk
    if nlos_var > 0.0:
        sd = math.sqrt(nlos_var / 2.0)
        for u in range(k):
            a, n = int(vstart[u]), int(vlen[u])
            g = rng.standard_normal((n, 2)) * sd
            H[u, a:a + n] += g[:, 0] + 1j * g[:, 1]
    H *= np.repeat(vis, L, axis=1)
    if symbols == "qpsk":
        S = qpsk(rng, (nrhs, k))
    elif symbols == "qam16":
        S = qam16(rng, (nrhs, k))
    else:
        raise ValueError(symbols)
    xi = k / (10.0 ** (snr_db / 10.0))
    return Drop(H=H, vr_start=vstart, vr_len=vlen, S=S, xi=float(xi), snr_db=float(snr_db),
                vr_mask=masks, n_sub=n_sub)


def make_multipath_drop(rng: np.random.Generator, *, nt: int = 2000, k: int = 30, nrhs: int = 0,
                        n_sub: int = 20, p_vis: float = 0.35, n_paths: int = 5, fc: float = 100e9,
                        r_lo: float = 1.0, r_hi: float = 50.0, snr_db: float = 0.0,
                        nlos_gain: float = 0.1) -> Drop:
    """Draw one drop of the simulation setting of the paper: the near-field
    multipath channel of Sec. II (LoS path plus n_paths - 1 scatterers, each
    a spherical-wave array response with phases relative to the array
    centre, scaled by sqrt(Nt / L_k)) on a ULA along the x axis with antenna
    n at (n d, 0), n = -(Nt-1)/2 .. (Nt-1)/2, times the Bernoulli subarray
    indicator. Each row is normalised to unit norm, so the per-user SNR
    rho ||h_k||^2 / sigma^2 is the same for every user (the power control
    of the simulation section), and xi = sigma^2 / rho = 1 / SNR.

    Choices the paper leaves open: users and scatterers at distances
    U[r_lo, r_hi] m and angles U[30, 150] degrees from the array axis (in
    front of it); gains beta_{k,1} ~ CN(0, 1) for the LoS path and
    CN(0, nlos_gain) for the others. Draw order: per user its path
    distances, angles and gains (LoS first), then the visibility matrix,
    then the symbols (nrhs QPSK vectors; nrhs = 0 for S = I_K work)."""
    if nt % n_sub or not 1 <= n_sub <= 64:
        raise ValueError("nt must be a multiple of n_sub, 1 <= n_sub <= 64")
    lam = C_LIGHT / fc
    d = lam / 2.0
    pos = (np.arange(nt) - (nt - 1) / 2.0) * d
    Hbar = np.zeros((k, nt), dtype=np.complex128)
    for u in range(k):
        r = rng.uniform(r_lo, r_hi, size=n_paths)
        th = np.deg2rad(rng.uniform(30.0, 150.0, size=n_paths))
        var = np.full(n_paths, nlos_gain)
        var[0] = 1.0
        g = (rng.standard_normal(n_paths) + 1j * rng.standard_normal(n_paths)) * np.sqrt(var / 2.0)
        for l in range(n_paths):
            dn = np.sqrt(r[l] ** 2 + pos ** 2 - 2.0 * pos * r[l] * np.cos(th[l]))
            Hbar[u] += g[l] * np.exp(-2j * np.pi * (dn - r[l]) / lam) / np.sqrt(nt)
        Hbar[u] *= np.sqrt(nt / n_paths)
    L = nt // n_sub
    vis = rng.random((k, n_sub)) < p_vis
    masks = np.array([sum(1 << s for s in range(n_sub) if vis[u, s]) for u in range(k)], dtype=np.uint64)
    vstart, vlen = mask_hulls(masks, nt, n_sub)
    H = Hbar * np.repeat(vis, L, axis=1)
    nrm = np.linalg.norm(H, axis=1)
    H[nrm > 0] /= nrm[nrm > 0, None]
    S = qpsk(rng, (nrhs, k))
    xi = 1.0 / (10.0 ** (snr_db / 10.0))
    return Drop(H=H, vr_start=vstart, vr_len=vlen, S=S, xi=float(xi), snr_db=float(snr_db),
                vr_mask=masks, n_sub=n_sub)


def _rng(cfg: int, seed: int, drop: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, seed, drop])))


# Workload recipes (seven named shapes):
#   plain      - one instance, Nt=256, K=16, LoS only, one QPSK vector, SNR 10 dB
#   many_rhs   - one channel, Nt=1024, K=64, LoS + CN(0,0.1), 4096 QPSK vectors
#   uneven     - 512 drops, Nt in {512,1024,2048}, K in [16,128], 256 vectors each
#   adjoint    - 256 drops of Nt=1024, K=64 with 64 QPSK vectors, SNR 10 dB
#   large      - 64 drops of Nt=4096, K=256, 1024 16-QAM vectors, SNR 10 dB
#   subarray   - 64 drops of the simulation setting of the paper: Nt=2000 at
#                100 GHz in S=20 subarrays, each visible w.p. 0.35, K=30 users
#                at 1..50 m, SNR 0 dB; 256 QPSK vectors each
#   paper      - 256 drops of the same setting with the paper's near-field
#                multipath channel (L_k = 5 paths, unit-norm rows, xi = 1/SNR),
#                for precoding matrices (S = I_K, no symbol vectors)
WORKLOADS = {
    "plain": dict(cfg=0, seed=0),
    "many_rhs": dict(cfg=1, seed=1),
    "uneven": dict(cfg=2, seed=2),
    "adjoint": dict(cfg=3, seed=3),
    "large": dict(cfg=4, seed=4),
    "subarray": dict(cfg=5, seed=5),
    "paper": dict(cfg=6, seed=6),
}


def make_workload(name: str, *, drops: int | None = None, nrhs: int | None = None,
                  snr_db: float | None = None, nt: int | None = None,
                  k: int | None = None, seed: int | None = None,
                  p_vis: float | None = None) -> list[Drop]:
    """Build the drops of a named workload. ``drops``/``nrhs``/``nt``/``k``
    shrink it for tests (same recipe, smaller shape); ``seed`` overrides the
    recipe's seed; ``p_vis`` the subarray visibility probability (subarray
    workload only)."""
    w = WORKLOADS[name]
    cfg, sd = w["cfg"], (w["seed"] if seed is None else seed)
    out = []
    if name == "plain":
        n = nt or 256
        kk = k or 16
        rng = _rng(cfg, sd, 0)
        out.append(make_drop(rng, nt=n, k=kk, nrhs=nrhs or 1, vr_lo=n // 4, vr_hi=n // 2,
                             snr_db=10.0 if snr_db is None else snr_db))
    elif name == "many_rhs":
        n = nt or 1024
        kk = k or 64
        for dd in range(drops or 1):
            rng = _rng(cfg, sd, dd)
            out.append(make_drop(rng, nt=n, k=kk, nrhs=nrhs or 4096, vr_lo=n // 4, vr_hi=n // 2,
                                 snr_db=10.0 if snr_db is None else snr_db, nlos_var=0.1))
    elif name == "uneven":
        for dd in range(drops or 512):
            rng = _rng(cfg, sd, dd)
            n = nt or int(rng.choice([512, 1024, 2048]))
            kk = k or int(rng.integers(16, 129))
            snr = float(rng.uniform(0.0, 20.0)) if snr_db is None else snr_db
            out.append(make_drop(rng, nt=n, k=kk, nrhs=nrhs or 256, vr_lo=n // 8, vr_hi=n // 2,
                                 snr_db=snr, nlos_var=0.1))
    elif name == "adjoint":
        n = nt or 1024
        kk = k or 64
        for dd in range(drops or 256):
            rng = _rng(cfg, sd, dd)
            out.append(make_drop(rng, nt=n, k=kk, nrhs=nrhs or 64, vr_lo=n // 4, vr_hi=n // 2,
                                 snr_db=10.0 if snr_db is None else snr_db, nlos_var=0.1))
    elif name == "large":
        n = nt or 4096
        kk = k or 256
        for dd in range(drops or 64):
            rng = _rng(cfg, sd, dd)
            out.append(make_drop(rng, nt=n, k=kk, nrhs=nrhs or 1024, vr_lo=n // 16, vr_hi=n // 4,
                                 snr_db=10.0 if snr_db is None else snr_db, nlos_var=0.1,
                                 symbols="qam16"))
    elif name == "subarray":
        n = nt or 2000
        kk = k or 30
        for dd in range(drops or 64):
            rng = _rng(cfg, sd, dd)
            out.append(make_subarray_drop(rng, nt=n, k=kk, nrhs=nrhs or 256, n_sub=20,
                                          p_vis=0.35 if p_vis is None else p_vis,
                                          snr_db=0.0 if snr_db is None else snr_db))
    elif name == "paper":
        for dd in range(drops or 256):
            rng = _rng(cfg, sd, dd)
            out.append(make_multipath_drop(rng, nt=nt or 2000, k=k or 30, nrhs=nrhs or 0,
                                           p_vis=0.35 if p_vis is None else p_vis,
                                           snr_db=0.0 if snr_db is None else snr_db))
    else:
        raise KeyError(name)
    return out
