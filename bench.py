#!/usr/bin/env python3
"""Throughput benchmark: precoded vectors/s on one MI355X.

Workload: one channel drop (Nt = 1024 antennas, K = 64 users, VR lengths
uniform in [256, 512] at uniform starts, LoS spherical wave at 28 GHz plus
CN(0, 0.1) scattering on the VR entries) with 4096 QPSK symbol vectors
sharing it, SNR 10 dB (xi = K / SNR), complex64, relative-residual
tolerance 1e-5. Inputs are synthetic and resident in HBM before timing.

One step = the hot path over the whole batch: the forward solve of all
4096 vectors with the chosen variant (VR-OAHK by default) and the
implicit-differentiation adjoint solve with gradient assembly. The plan
(VR graph, colours, tiles) and the row norms / tile packing of the channel
are built once before timing. The forward solve kernel is timed live with
HIP events on the stream it runs on (the roofline's "achieved").

Prints one JSON line. Extra fields: per-variant forward rates, the plain
single-instance rate (one vector per launch), accuracy against the FP64
Cholesky RZF, and the FP64 oracle timed on the host (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "precoded vectors/s at rel err<=1e-4 vs FP64 RZF; batched+adjoint vs plain"
PEAK_MFMA_F32 = 157.3e12     # dense FP32 matrix-core peak, MI355X
PEAK_VALU_F32 = 78.6e12      # FP32 vector FMA without packed-FP32 instructions
PEAK_HBM = 8.0e12


def algorithmic_flops(variant, band, band_f, band_v, iters, k):
    """Real flops of one solve per the band structure (8 per complex MAC,
    Table I's counting with |Gamma| taken per user): GRK / VR-OGRK: a full
    banded residual per row update (the selection needs every residual)
    plus the row update; AHK: residual + aggregation; VR-OAHK: residual
    check, F half-step, V residual and V aggregation. `iters` = sum over
    vectors of the updates each vector made."""
    if variant in ("grk", "vr_ogrk"):
        return iters * 8.0 * band * (1.0 + 1.0 / k)
    if variant == "ahk":
        return iters * 16.0 * band
    return iters * 8.0 * (band + band_f + 2.0 * band_v)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="vr_oahk", choices=["grk", "ahk", "vr_ogrk", "vr_oahk"])
    ap.add_argument("--engine", default="auto", choices=["auto", "vector", "mfma"])
    ap.add_argument("--nrhs", type=int, default=4096)
    ap.add_argument("--snr", type=float, default=10.0)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--tile-waves", type=int, default=0, choices=[0, 8, 16])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path has no cross-GPU exchange "
              "(drops shard with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2501_10689_amd import vrk

    dev = torch.device("cuda:0")
    d = synth.make_workload("many_rhs", nrhs=args.nrhs, snr_db=args.snr)[0]
    B, K, N = d.nrhs, d.k, d.nt
    c64 = torch.complex64
    H = torch.from_numpy(d.H).to(c64).to(dev)
    S = torch.from_numpy(d.S).to(c64).to(dev)
    X = torch.zeros((B, N), dtype=c64, device=dev)
    V = torch.zeros((B, K), dtype=c64, device=dev)
    g = np.random.default_rng(12345)
    Gh = (g.standard_normal((B, N)) + 1j * g.standard_normal((B, N))) * (1.0 / B)
    GX = torch.from_numpy(Gh).to(c64).to(dev)
    GH = torch.zeros_like(H)
    GS = torch.zeros_like(S)
    gxi = torch.zeros(1, dtype=torch.float64, device=dev)
    opts = vrk.options(variant=args.variant, dtype="c64", engine=args.engine, tol=args.tol,
                       tile_waves=args.tile_waves)
    plan = vrk.Plan([vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S, X, V, GX, GH, GS, gxi)], opts)
    eng = plan.query(0, vrk.Q_ENGINE)
    engine = {1: "vector", 2: "mfma"}[int(eng[0])]
    stats = plan.stats_buffers()
    stats_adj = plan.stats_buffers()
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.solve(stream=stream, stats=stats)
        if ev is not None:
            ev[1].record(stream)
        plan.solve_adjoint(stream=stream, stats=stats_adj)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for i in range(args.steps):
        step(evs[i])
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    solve_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    value = B / (ms_step * 1e-3)

    # accuracy of this run vs the FP64 Cholesky RZF (the oracle's plain definition)
    import oracle
    Xr, Vr = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    Xg = X.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(Xg - Xr, axis=1) / np.linalg.norm(Xr, axis=1)
    it = stats[0].cpu().numpy()
    fl = stats[2].cpu().numpy()
    flf = plan.query(0, vrk.Q_FSET)
    vl = np.asarray(d.vr_len, dtype=np.int64)
    band = float(vl.sum())
    band_f = float(vl[flf].sum())
    band_v = band - band_f
    iters_total = float(it.sum())
    flops = algorithmic_flops(args.variant, band, band_f, band_v, iters_total, K)
    achieved = flops / (solve_ms * 1e-3)
    if engine == "mfma":
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_MFMA_F32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_F32, "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_F32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_F32, "traffic": None}
    roof["kernel"] = "solve (%s engine, %s)" % (engine, args.variant)
    roof["kernel_ms"] = solve_ms
    roof["flops_per_launch"] = flops
    roof["unit_of_work"] = "vector-iteration"
    roof["units_per_launch"] = iters_total

    out = {
        "metric": METRIC, "value": value, "unit": "vectors/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single channel, many symbols: Nt=1024, K=64, VR U[256,512], "
                               "LoS+CN(0,0.1), %d QPSK vectors, SNR %g dB, tol %g; fwd+adjoint"
                               % (B, args.snr, args.tol),
                   "variant": args.variant, "engine": engine, "tile_waves": int(eng[2]),
                   "nrhs": B, "nt": N, "k": K},
        "roofline": roof,
        "accuracy": {"max_rel_err": float(err.max()), "mean_rel_err": float(err.mean()),
                     "all_converged": bool(np.all(fl == 1)), "mean_iters": float(it.mean()),
                     "max_iters": int(it.max())},
    }

    # per-variant forward rates (same workload, same engine choice)
    if not args.no_variants:
        rates = {}
        for var in ("grk", "ahk", "vr_ogrk", "vr_oahk"):
            Xv = torch.zeros_like(X)
            Vv = torch.zeros_like(V)
            pv = vrk.Plan([vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S, Xv, Vv)],
                          vrk.options(variant=var, dtype="c64", engine=args.engine, tol=args.tol,
                                      tile_waves=args.tile_waves))
            sv = pv.stats_buffers()
            pv.solve(stream=stream, stats=sv)
            torch.cuda.synchronize()
            reps = 3 if var in ("grk", "vr_ogrk") else 10
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                pv.solve(stream=stream, stats=sv)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            e2 = np.linalg.norm(Xv.cpu().numpy() - Xr, axis=1) / np.linalg.norm(Xr, axis=1)
            rates[var] = {"vectors_per_s": B / (ms * 1e-3), "ms": ms, "max_rel_err": float(e2.max()),
                          "mean_iters": float(sv[0].float().mean().item())}
            del pv
        out["variants_fwd"] = rates

    # plain single-instance solver: one vector per launch, fwd + adjoint
    if not args.no_plain:
        n_plain = 128
        S1 = torch.zeros((1, K), dtype=c64, device=dev)
        X1 = torch.zeros((1, N), dtype=c64, device=dev)
        V1 = torch.zeros((1, K), dtype=c64, device=dev)
        G1 = torch.zeros((1, N), dtype=c64, device=dev)
        GH1 = torch.zeros_like(H)
        GS1 = torch.zeros((1, K), dtype=c64, device=dev)
        gx1 = torch.zeros(1, dtype=torch.float64, device=dev)
        p1 = vrk.Plan([vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S1, X1, V1, G1, GH1, GS1, gx1)],
                      vrk.options(variant=args.variant, dtype="c64", engine="vector", tol=args.tol))
        errs = []
        for i in range(3):
            S1.copy_(S[i:i + 1])
            G1.copy_(GX[i:i + 1])
            p1.solve(stream=stream)
            p1.solve_adjoint(stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for i in range(n_plain):
            S1.copy_(S[i:i + 1])
            G1.copy_(GX[i:i + 1])
            p1.solve(stream=stream)
            p1.solve_adjoint(stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        x1 = X1.cpu().numpy()[0]
        i = n_plain - 1
        errs.append(float(np.linalg.norm(x1 - Xr[i]) / np.linalg.norm(Xr[i])))
        plain_rate = n_plain / (ms * 1e-3)
        out["plain"] = {"vectors_per_s": plain_rate, "engine": "vector, one vector per launch",
                        "sample": n_plain, "rel_err_last": errs[-1]}
        out["speedup_vs_plain"] = value / plain_rate

    # FP64 oracle on the host: the same workload (forward iterations with the
    # same variant and tolerance, plus the closed-form gradient), sampled
    if not args.no_cpu_baseline:
        n_cpu = min(B, 4096)
        Ss = d.S[:n_cpu]
        t = time.perf_counter()
        oracle.solve_batch(d.H, d.vr_start, d.vr_len, Ss, d.xi, variant=args.variant, tol=args.tol)
        oracle.rzf_grad(d.H, d.vr_start, d.vr_len, Ss, d.xi, Gh[:n_cpu])
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": n_cpu / dt, "unit": "vectors/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": "%d of the %d vectors: FP64 %s iterations to tol %g "
                                         "(OpenMP over vectors) + closed-form gradient"
                                         % (n_cpu, B, args.variant, args.tol)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
