#!/usr/bin/env python3
"""Throughput benchmark: precoded vectors/s on one MI355X.

Default workload (--workload large): 64 channel drops of Nt = 4096 antennas
and K = 256 users (VR lengths uniform in [256, 1024] at uniform starts, LoS
spherical wave at 28 GHz plus CN(0, 0.1) scattering on the VR entries), each
with 1024 16-QAM symbol vectors, SNR 10 dB (xi = K / SNR), complex64,
relative-residual tolerance 1e-5, VR-OAHK forward plus adjoint in one
batched launch each. The other workloads:
  many_rhs one drop Nt 1024, K 64, VR U[256, 512], 4096 QPSK vectors, SNR 10 dB
  uneven   512 drops, Nt in {512, 1024, 2048}, K in [16, 128], VR U[Nt/8, Nt/2],
           256 QPSK vectors each, SNR U[0, 20] dB (one launch for all drops)
  adjoint  256 drops of Nt 1024, K 64, VR U[256, 512], 64 QPSK vectors, SNR 10 dB
  plain    one drop Nt 256, K 16, LoS, VR U[64, 128], one QPSK vector, complex128,
           tolerance 1e-10
  subarray 64 drops of the paper's simulation setting: Nt 2000 at 100 GHz in 20
           subarrays, each visible to each user w.p. 0.35, K 30, SNR 0 dB,
           256 QPSK vectors each (VRs are unions of subarrays)
  precoder the adjoint workload's 256 drops with S = I_K: each drop's RZF precoding
           matrix, its effective channel, beta and per-user spectral efficiency
           (metric: precoding matrices/s; see run_precoder)
  paper_precoder  the same for 256 drops of the paper's simulation setting (Nt 2000,
           100 GHz, 20 subarrays visible w.p. 0.35, K 30, five near-field paths, SNR 0 dB)
Inputs are synthetic and resident in HBM before timing.

One step = the hot path over the whole batch: what the binding derives from
the channels (row norms, channel and Gram tiles: vrk_plan_refresh, since the
channel is an input of the differentiated step), the forward solve of every
vector with the chosen variant (VR-OAHK by default) and the
implicit-differentiation adjoint (b = H g, adjoint solve, gradient
assembly). The plan (VR graph, colours, tiles) is built once before timing.
The step is captured once into a HIP graph and the timed value comes from
replays of it (--eager: from eager launches); the rate without the refresh
(one channel serving many symbol batches) is reported beside it. The forward
solve kernel is timed live with HIP events on the stream it runs on, in an
eager loop before the replays; its algorithmic flops over that time are the
roofline's "achieved".

Prints one JSON line. Extra fields: per-variant forward rates (many_rhs), the
plain single-instance rate (one vector per launch, launches replayed from a
HIP graph) and the plain configuration's microseconds per solve next to the
oracle's, accuracy of every vector against the FP64 Cholesky RZF, and the
FP64 oracle timed on the host (cpu_baseline, with its Cholesky-RZF,
VR-OAHK and GRK legs at all threads and one thread).
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
PEAK_VALU_F64 = 78.6e12

WORKLOADS = {
    "many_rhs": "single channel, many symbols: Nt=1024, K=64, VR U[256,512], LoS+CN(0,0.1), "
                "4096 QPSK vectors, SNR 10 dB, tol 1e-5; fwd+adjoint",
    "uneven": "uneven batch: 512 drops, Nt in {512,1024,2048}, K U[16,128], VR U[Nt/8,Nt/2], "
              "256 QPSK vectors each, SNR U[0,20] dB, tol 1e-5; fwd+adjoint",
    "adjoint": "adjoint: 256 drops of Nt=1024, K=64, VR U[256,512], 64 QPSK vectors each, "
               "SNR 10 dB, tol 1e-5; fwd+adjoint",
    "large": "large fwd+bwd: 64 drops of Nt=4096, K=256, VR U[256,1024], 1024 16-QAM vectors each, "
             "SNR 10 dB, tol 1e-5; fwd+adjoint",
    "plain": "plain single instance: Nt=256, K=16, LoS, VR U[64,128], one QPSK vector, SNR 10 dB, "
             "complex128, tol 1e-10; fwd+adjoint",
    "subarray": "subarray VRs (simulation setting of the paper): 64 drops of Nt=2000 at 100 GHz in S=20 "
                "subarrays, each visible w.p. 0.35, K=30 at 1..50 m, LoS+CN(0,0.1) on visible antennas, "
                "256 QPSK vectors each, SNR 0 dB, tol 1e-5; fwd+adjoint",
    "paper_precoder": "RZF precoding matrices in the paper's simulation setting: 256 drops of Nt=2000 at 100 GHz, "
                      "S=20 subarrays visible w.p. 0.35, K=30 at 1..50 m, L_k=5 near-field paths, unit-norm "
                      "rows, SNR 0 dB (xi = 1), S = I_K, tol 1e-5; solve + effective channel + beta + per-user "
                      "spectral efficiency",
    "precoder": "RZF precoding matrices: 256 drops of Nt=1024, K=64, VR U[256,512], S = I_K, SNR 10 dB, "
                "tol 1e-5; solve + effective channel + beta + per-user spectral efficiency",
}


def time_bind(plan, stream, reps=11):
    """Median time of vrk_plan_bind on the stream (plan tables to the
    workspace, row norms, tile packing and Gram tiles: the per-channel setup
    that precedes the solves), in ms, over reps binds after a warm-up."""
    import statistics

    import torch
    plan.bind(stream)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.bind(stream)
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def run_precoder(args):
    """One step = every drop's precoding matrix (the solve on S = I_K, rows of X
    = columns of F) and its link metrics (vrk_link_metrics). Accuracy: NMSE of
    beta F against the FP64 Cholesky RZF's, and the largest per-user rate
    difference. cpu_baseline: the oracle's FP64 iterations on S = I_K plus its
    link metrics on a bounded sample of drops."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2501_10689_amd import vrk

    dev = torch.device("cuda:0")
    wl = args.workload
    drops = synth.make_workload("paper" if wl == "paper_precoder" else "adjoint", snr_db=args.snr)
    tol = args.tol if args.tol is not None else 1e-5
    specs, E, R, Bt = [], [], [], []
    for d in drops:
        H = torch.from_numpy(d.H).to(torch.complex64).to(dev)
        S = torch.eye(d.k, dtype=torch.complex64, device=dev)
        X = torch.zeros((d.k, d.nt), dtype=torch.complex64, device=dev)
        specs.append(vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S, X, vr_mask=d.vr_mask, n_sub=d.n_sub))
        E.append(torch.zeros((d.k, d.k), dtype=torch.complex64, device=dev))
        R.append(torch.zeros(d.k, dtype=torch.float64, device=dev))
        Bt.append(torch.zeros(1, dtype=torch.float64, device=dev))
    opts = vrk.options(variant=args.variant, dtype="c64", engine=args.engine, tol=tol,
                       tile_waves=args.tile_waves, persistent=args.persistent)
    plan = vrk.Plan(specs, opts)
    # sigma^2 / rho of the rates: 1 / SNR (the regulariser is K / SNR on the
    # adjoint drops, 1 / SNR on the paper's setting)
    noise = [10.0 ** (-d.snr_db / 10.0) for d in drops]
    eng = plan.query(0, vrk.Q_ENGINE)
    engine = {1: "vector", 2: "mfma"}[int(eng[0])]
    stats = plan.stats_buffers()
    stream = torch.cuda.current_stream(dev)
    bind_ms = time_bind(plan, stream)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.solve(stream=stream, stats=stats)
        if ev is not None:
            ev[1].record(stream)
        plan.link_metrics(E, R, Bt, noise, stream=stream)

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
    ms_eager = ms_step
    if not args.eager:
        # replays of the step captured in a HIP graph (the output table is
        # already in the workspace from the eager calls, so the capture holds
        # kernels only)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.solve(stats=stats)
            plan.link_metrics(E, R, Bt, noise)
        for _ in range(max(1, args.warmup)):
            graph.replay()
        torch.cuda.synchronize()
        t0.record(stream)
        for i in range(args.steps):
            graph.replay()
        t1.record(stream)
        torch.cuda.synchronize()
        ms_step = t0.elapsed_time(t1) / args.steps
    value = len(drops) / (ms_step * 1e-3)

    it_all = stats[0].cpu().numpy()
    worst_nmse, worst_rate, flops, base = 0.0, 0.0, 0.0, 0
    for j, (d, sp) in enumerate(zip(drops, specs)):
        Xo = oracle.precoder(d.H, d.vr_start, d.vr_len, d.xi)
        _, bo, ro = oracle.link_metrics(d.H, d.vr_start, d.vr_len, noise[j], Xo)
        Xg = sp.X.cpu().numpy().astype(np.complex128)
        bg = float(Bt[j].cpu().numpy()[0])
        worst_nmse = max(worst_nmse, oracle.nmse(bo * Xo, bg * Xg))
        worst_rate = max(worst_rate, float(np.max(np.abs(R[j].cpu().numpy() - ro))))
        fset = plan.query(j, vrk.Q_FSET)
        vl = np.asarray(d.vr_len, dtype=np.int64)
        if d.vr_mask is not None:   # the visible antennas of each user, not its hull
            vl = np.array([bin(int(m)).count("1") * (d.nt // d.n_sub) for m in d.vr_mask], dtype=np.int64)
        band, band_f = float(vl.sum()), float(vl[fset].sum())
        it = it_all[base:base + d.k]
        overlap = float(plan.query(j, vrk.Q_XOFF)[-1])
        flops += algorithmic_flops(engine, args.variant, band, band_f, band - band_f, overlap, float(it.sum()),
                                   float(d.k), d.k)
        base += d.k
    achieved = flops / (solve_ms * 1e-3)
    roof = {"bound": "mfma" if engine == "mfma" else "alu", "achieved": achieved / 1e12,
            "peak": (PEAK_MFMA_F32 if engine == "mfma" else PEAK_VALU_F32) / 1e12, "unit": "TFLOP/s",
            "frac": achieved / (PEAK_MFMA_F32 if engine == "mfma" else PEAK_VALU_F32), "traffic": None,
            "kernel": "solve on S = I_K (%s engine, %s)" % (engine, args.variant), "kernel_ms": solve_ms,
            "flops_per_launch": flops, "unit_of_work": "vector-iteration", "units_per_launch": float(it_all.sum())}
    out = {
        "metric": "RZF precoding matrices/s with link metrics, NMSE <= 1e-4 vs FP64 RZF",
        "value": value, "unit": "matrices/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "timing": "eager launches" if args.eager else
                  "HIP graph of the step, replayed (eager: %.4f ms per step)" % ms_eager,
        "config": {"workload": WORKLOADS[wl], "variant": args.variant, "engine": engine,
                   "tile_waves": int(eng[2]), "entries_per_thread": int(eng[6]), "drops": len(drops),
                   "vectors": int(sum(d.k for d in drops)), "tol": tol},
        "roofline": roof,
        "bind_ms": bind_ms,
        "matrices_per_s_with_bind": len(drops) / ((ms_step + bind_ms) * 1e-3),
        "accuracy": {"max_nmse": worst_nmse, "max_rate_diff_bits": worst_rate,
                     "mean_iters": float(it_all.mean()), "max_iters": int(it_all.max())},
    }
    if not args.no_cpu_baseline:
        # drops in order, cycling when one pass takes less than the budget
        budget, n_cpu, t_cpu = 10.0, 0, 0.0
        while t_cpu <= budget:
            d = drops[n_cpu % len(drops)]
            t = time.perf_counter()
            Xc = oracle.solve_batch(d.H, d.vr_start, d.vr_len, np.eye(d.k, dtype=np.complex128), d.xi,
                                    variant=args.variant, tol=tol, masks=d.vr_mask, n_sub=d.n_sub)["X"]
            oracle.link_metrics(d.H, d.vr_start, d.vr_len, 10.0 ** (-d.snr_db / 10.0), Xc)
            t_cpu += time.perf_counter() - t
            n_cpu += 1
        out["cpu_baseline"] = {"value": n_cpu / t_cpu, "unit": "matrices/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": "%d drop solves (drops taken in order, %d distinct of %d; %.1f s): FP64 "
                                         "%s iterations on S = I_K to tol %g (OpenMP over vectors) + link metrics"
                                         % (n_cpu, min(n_cpu, len(drops)), len(drops), t_cpu, args.variant, tol)}
    print(json.dumps(out), flush=True)


def algorithmic_flops(engine, variant, band, band_f, band_v, overlap, iters, vectors, k):
    """Real flops of one solve launch, 8 per complex multiply-add.

    Vector engine (the paper's steps, Table I's counting with |Gamma| taken
    per user): GRK / VR-OGRK a full banded residual per row update plus the
    row update; AHK residual + aggregation; VR-OAHK residual check, F
    half-step, V residual and V aggregation.

    MFMA engine (dual-space iteration): per vector-iteration the Gram
    products over the users' overlap sets, sum_i |X_i| = `overlap` complex
    multiply-adds for the aggregated variants (the F and V columns of M),
    |X_pick| (on average overlap / K) for the greedy ones; once per vector
    x = H^H q (band) and the fresh residual s - M q (overlap).

    `iters` = sum over vectors of the iterations each vector made."""
    if engine == "mfma":
        per_it = overlap / k if variant in ("grk", "vr_ogrk") else overlap
        return 8.0 * (iters * per_it + vectors * (band + overlap))
    if variant in ("grk", "vr_ogrk"):
        return iters * 8.0 * band * (1.0 + 1.0 / k)
    if variant == "ahk":
        return iters * 16.0 * band
    return iters * 8.0 * (band + band_f + 2.0 * band_v)


# Kernel sources whose rocprofv3 counters the committed traffic files hold.
TRAFFIC_SOURCES = ["paper_2501_10689_amd/csrc/mfma_engine.hip", "paper_2501_10689_amd/csrc/wave_engine.hip",
                   "paper_2501_10689_amd/csrc/device_common.h", "paper_2501_10689_amd/csrc/vrk_desc.h",
                   "paper_2501_10689_amd/csrc/kernels.h"]


def measured_traffic(workload, kernel_prefix):
    """HBM bytes per launch of the solve kernel from profiles/traffic_solve_<workload>.txt
    (FETCH_SIZE and WRITE_SIZE per dispatch scaled by a plain copy's reading), or None
    when there is no such file, it covers another kernel instantiation, or the kernel
    sources changed since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "traffic_solve_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    if kv.get("source_sha256") != h.hexdigest() or not kv.get("kernel", "").startswith(kernel_prefix):
        return None
    return float(kv["hbm_bytes_per_launch"])


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_leg(drops, budget_s, work):
    """Runs work(drop) -> vectors over the drops in order (cycling) until
    budget_s of wall time is spent; returns (vectors/s, vectors, drop calls,
    seconds)."""
    n_vec, calls, t_all = 0, 0, 0.0
    while t_all <= budget_s:
        d = drops[calls % len(drops)]
        t = time.perf_counter()
        n_vec += work(d)
        t_all += time.perf_counter() - t
        calls += 1
    return n_vec / t_all, n_vec, calls, t_all


def cpu_baseline(drops, variant, tol, wl, threads):
    """The FP64 oracle timed on the host, on bounded samples of the same
    workload: the same work as one GPU step (the variant's iterations plus the
    closed-form gradient), and the legs of the CPU baseline plan (Cholesky
    RZF, reference VR-OAHK, reference GRK), each with all threads and with
    one thread."""
    import numpy as np

    import oracle
    gcpu = np.random.default_rng(7)
    cap = 256 if wl == "large" else None

    def sub(d, n=None):
        n = d.nrhs if n is None else min(n, d.nrhs)
        return d.S[:n], dict(masks=d.vr_mask, n_sub=d.n_sub)

    def step_work(d):
        Ss, mk = sub(d, cap)
        G = (gcpu.standard_normal((len(Ss), d.nt)) + 1j * gcpu.standard_normal((len(Ss), d.nt))) / d.nrhs
        oracle.solve_batch(d.H, d.vr_start, d.vr_len, Ss, d.xi, variant=variant, tol=tol, **mk)
        oracle.rzf_grad(d.H, d.vr_start, d.vr_len, Ss, d.xi, G, **mk)
        return len(Ss)

    def chol_work(d):
        Ss, mk = sub(d)
        oracle.rzf(d.H, d.vr_start, d.vr_len, Ss, d.xi, **mk)
        return len(Ss)

    def iter_work(var, n):
        def f(d):
            Ss, mk = sub(d, n)
            oracle.solve_batch(d.H, d.vr_start, d.vr_len, Ss, d.xi, variant=var, tol=tol, **mk)
            return len(Ss)
        return f

    out = {}
    nthreads = threads
    oracle.set_num_threads(nthreads)
    v, n, c, t = timed_leg(drops, 8.0, step_work)
    out["step"] = (v, "%d vectors in %d drop solves (drops in order, %d distinct of %d; %.1f s): FP64 %s "
                   "iterations to tol %g + closed-form gradient, %d threads"
                   % (n, c, min(c, len(drops)), len(drops), t, variant, tol, nthreads))
    legs = {}
    # per leg: (work with all threads, work with one thread, seconds); the
    # greedy leg costs about a hundred times the aggregated one per vector
    grk_n = 16 if wl == "large" else 64
    plan_legs = (("cholesky_rzf", chol_work, chol_work, 3.0),
                 ("vr_oahk", iter_work("vr_oahk", cap), iter_work("vr_oahk", 32), 3.0),
                 ("grk", iter_work("grk", grk_n * nthreads), iter_work("grk", 2), 4.0))
    for label, w_all, w_one, budget in plan_legs:
        row = {}
        for th, w, bud in ((nthreads, w_all, budget), (1, w_one, budget / 2)):
            oracle.set_num_threads(th)
            v, n, c, t = timed_leg(drops, bud, w)
            row["vectors_per_s_%dthreads" % th] = v
            row["sample_%dthreads" % th] = "%d vectors, %d drop calls, %.1f s" % (n, c, t)
        legs[label] = row
    oracle.set_num_threads(nthreads)
    return out["step"], legs


def plain_leg(d0, sp0, cdt, variant, tol, n_plain, stream):
    """The plain single-instance GPU solver: one vector per launch (vector
    engine), forward + adjoint, on n_plain rows of the first drop. One plan per
    vector (its S, X, V, GX rows are views into the batch buffers) so that the
    n_plain solves are captured once into a HIP graph and replayed: no host
    work between the launches. Returns (vectors/s, us per vector, the last
    vector's X row)."""
    import torch

    from paper_2501_10689_amd import vrk
    dev = sp0.H.device
    plans = []
    for i in range(n_plain):
        sp = vrk.ProblemSpec(sp0.H, d0.vr_start, d0.vr_len, d0.xi, sp0.S[i:i + 1], sp0.X[i:i + 1].clone(),
                             sp0.V[i:i + 1].clone(), sp0.GX[i:i + 1], torch.zeros_like(sp0.H),
                             torch.zeros((1, d0.k), dtype=cdt, device=dev),
                             torch.zeros(1, dtype=torch.float64, device=dev),
                             vr_mask=d0.vr_mask, n_sub=d0.n_sub)
        plans.append(vrk.Plan([sp], vrk.options(variant=variant, dtype="c128" if cdt == torch.complex128 else "c64",
                                                engine="vector", tol=tol)))
    for p in plans:
        p.solve(stream=stream)
        p.solve_adjoint(stream=stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for p in plans:
            p.solve()
            p.solve_adjoint()
    graph.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    reps = 3
    a.record(stream)
    for _ in range(reps):
        graph.replay()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return n_plain / (ms * 1e-3), ms * 1e3 / n_plain, plans[-1].probs[0].X


def plain_c1(stream):
    """The plain single-instance configuration itself (Nt 256, K 16, LoS, one
    QPSK vector, complex128, tolerance 1e-10): microseconds per forward solve
    on the GPU (graph replays of one-vector launches) per variant, next to the
    FP64 oracle's time per vector on the host (one thread: a single vector)."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2501_10689_amd import vrk
    d = synth.make_workload("plain")[0]
    dev = torch.device("cuda:0")
    H = torch.from_numpy(d.H).to(dev)
    S = torch.from_numpy(d.S).to(dev)
    Xr, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi)
    out = {}
    for var in ("grk", "ahk", "vr_oahk"):
        us = {}
        for waves in (1, 4):   # the single-wave form (chosen for this size) and the four-wave form
            X = torch.zeros((1, d.nt), dtype=torch.complex128, device=dev)
            V = torch.zeros((1, d.k), dtype=torch.complex128, device=dev)
            plan = vrk.Plan([vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S, X, V)],
                            vrk.options(variant=var, dtype="c128", engine="vector", tol=1e-10, tile_waves=waves))
            st = plan.stats_buffers()
            plan.solve(stream=stream, stats=st)
            torch.cuda.synchronize()
            n = 64
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                for _ in range(n):
                    plan.solve(stats=st)
            graph.replay()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            graph.replay()
            b.record(stream)
            torch.cuda.synchronize()
            us[waves] = a.elapsed_time(b) * 1e3 / n
        err = float(np.linalg.norm(X.cpu().numpy()[0] - Xr[0]) / np.linalg.norm(Xr[0]))
        reps, t = 0, 0.0
        while t < 0.3:
            t0 = time.perf_counter()
            oracle.solve(d.H, d.vr_start, d.vr_len, d.S[0], d.xi, variant=var, tol=1e-10)
            t += time.perf_counter() - t0
            reps += 1
        out[var] = {"gpu_us_per_solve": us[1], "gpu_us_per_solve_four_wave": us[4],
                    "oracle_us_per_solve": t * 1e6 / reps, "iters": int(st[0].cpu()[0]), "rel_err": err}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="vr_oahk", choices=["grk", "ahk", "vr_ogrk", "vr_oahk"])
    ap.add_argument("--engine", default="auto", choices=["auto", "vector", "mfma"])
    ap.add_argument("--snr", type=float, default=None)
    ap.add_argument("--p-vis", type=float, default=None,
                    help="subarray workload: visibility probability of each subarray (default 0.35)")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--tile-waves", type=int, default=0, choices=[0, 1, 4, 8, 16],
                    help="MFMA engine: waves per tile (8, 16); vector engine: waves per vector (1, 4); 0 auto")
    ap.add_argument("--persistent", type=int, default=0, choices=[0, 1])
    ap.add_argument("--wave-tiles", type=int, default=0, choices=[-1, 0, 1, 2, 4, 8],
                    help="MFMA engine, AHK / VR-OAHK: waves per wave-owned tile (-1 block tiles, 0 auto)")
    ap.add_argument("--autotune", action="store_true", help="pick engine/tiles with vrk_autotune first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches instead of replays of the step captured in a HIP graph")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after timing, copy a device buffer of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path has no cross-GPU exchange "
              "(drops shard with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload in ("precoder", "paper_precoder"):
        run_precoder(args)
        return

    import numpy as np
    import torch

    import synth
    from paper_2501_10689_amd import vrk

    dev = torch.device("cuda:0")
    wl = args.workload
    c128 = wl == "plain"
    cdt = torch.complex128 if c128 else torch.complex64
    dname = "c128" if c128 else "c64"
    tol = args.tol if args.tol is not None else (1e-10 if c128 else 1e-5)
    engine_opt = "vector" if c128 else args.engine
    if args.p_vis is not None and wl != "subarray":
        sys.exit("--p-vis applies to the subarray workload only")
    drops = synth.make_workload(wl, snr_db=args.snr, **({"p_vis": args.p_vis} if args.p_vis is not None else {}))
    gen = torch.Generator(device=dev)
    gen.manual_seed(12345)
    specs = []
    for d in drops:
        H = torch.from_numpy(d.H).to(cdt).to(dev)
        S = torch.from_numpy(d.S).to(cdt).to(dev)
        X = torch.zeros((d.nrhs, d.nt), dtype=cdt, device=dev)
        V = torch.zeros((d.nrhs, d.k), dtype=cdt, device=dev)
        GX = (torch.randn((d.nrhs, d.nt), dtype=cdt, device=dev, generator=gen) / d.nrhs)
        specs.append(vrk.ProblemSpec(H, d.vr_start, d.vr_len, d.xi, S, X, V, GX, torch.zeros_like(H),
                                     torch.zeros_like(S), torch.zeros(1, dtype=torch.float64, device=dev),
                                     vr_mask=d.vr_mask, n_sub=d.n_sub))
    B = sum(d.nrhs for d in drops)
    opts = vrk.options(variant=args.variant, dtype=dname, engine=engine_opt, tol=tol,
                       tile_waves=args.tile_waves, persistent=args.persistent, wave_tiles=args.wave_tiles)
    tuned_ms = None
    if args.autotune:
        opts, tuned_ms = vrk.autotune(specs, opts, reps=3)
    plan = vrk.Plan(specs, opts)
    eng = plan.query(0, vrk.Q_ENGINE)
    engine = {1: "vector", 2: "mfma"}[int(eng[0])]
    stats = plan.stats_buffers()
    stats_adj = plan.stats_buffers()
    stream = torch.cuda.current_stream(dev)
    bind_ms = time_bind(plan, stream)

    # One step: what the binding derives from the channel (row norms, tiles,
    # Gram tiles: vrk_plan_refresh), the forward solve of every vector and the
    # adjoint (b = H g, adjoint solve, gradient assembly). The channel is an
    # input of the differentiated step, so its per-channel work is timed too.
    def step(ev=None, refresh=True):
        if refresh:
            plan.refresh(stream=stream)
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
    ms_eager = ms_step
    ms_reuse = None
    if not args.eager:
        # the step captured once into a HIP graph and replayed: the timed
        # value (the eager loop above gives the live per-launch solve time);
        # a second graph without the refresh gives the rate when one channel
        # serves many batches of symbols
        def replay_ms(refresh):
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                if refresh:
                    plan.refresh()
                plan.solve(stats=stats)
                plan.solve_adjoint(stats=stats_adj)
            for _ in range(max(1, args.warmup)):
                graph.replay()
            torch.cuda.synchronize()
            t0.record(stream)
            for _ in range(args.steps):
                graph.replay()
            t1.record(stream)
            torch.cuda.synchronize()
            return t0.elapsed_time(t1) / args.steps
        ms_step = replay_ms(True)
        ms_reuse = replay_ms(False)
    value = B / (ms_step * 1e-3)

    # accuracy of every vector vs the FP64 Cholesky RZF, and the flop counts
    import oracle
    it_all = stats[0].cpu().numpy()
    fl_all = stats[2].cpu().numpy()
    worst, errsum, flops, flops_primal, base = 0.0, 0.0, 0.0, 0.0, 0
    for j, (d, sp) in enumerate(zip(drops, specs)):
        Xr, _ = oracle.rzf(d.H, d.vr_start, d.vr_len, d.S, d.xi, masks=d.vr_mask, n_sub=d.n_sub)
        Xg = sp.X.cpu().numpy().astype(np.complex128)
        e = np.linalg.norm(Xg - Xr, axis=1) / np.linalg.norm(Xr, axis=1)
        worst = max(worst, float(e.max()))
        errsum += float(e.sum())
        fset = plan.query(j, vrk.Q_FSET)
        vl = np.asarray(d.vr_len, dtype=np.int64)
        if d.vr_mask is not None:   # the visible antennas of each user, not its hull
            vl = np.array([bin(int(m)).count("1") * (d.nt // d.n_sub) for m in d.vr_mask], dtype=np.int64)
        band, band_f = float(vl.sum()), float(vl[fset].sum())
        it = it_all[base:base + d.nrhs]
        overlap = float(plan.query(j, vrk.Q_XOFF)[-1])   # sum_i |X_i|
        args_f = (args.variant, band, band_f, band - band_f, overlap, float(it.sum()), float(d.nrhs), d.k)
        flops += algorithmic_flops(engine, *args_f)
        flops_primal += algorithmic_flops("vector", *args_f)
        base += d.nrhs
    achieved = flops / (solve_ms * 1e-3)
    if engine == "mfma":
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_MFMA_F32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_F32, "traffic": None}
    else:
        peak = PEAK_VALU_F64 if c128 else PEAK_VALU_F32
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None}
    if engine == "mfma":
        vid = {"grk": 0, "vr_ogrk": 0, "ahk": 1, "vr_oahk": 3}[args.variant]
        if int(eng[10]):
            kname = "void (anonymous namespace)::k_wave_solve<%d, %d, %d>" % (int(eng[10]), int(eng[11]), vid)
        else:
            kname = "void (anonymous namespace)::k_mfma_solve<%d, %d, %d, %s>" % (
                int(eng[2]), int(eng[6]), vid, "true" if int(eng[4]) else "false")
        roof["traffic"] = measured_traffic(wl, kname)
    roof["kernel"] = "forward solve (%s engine, %s)" % (engine, args.variant)
    roof["kernel_ms"] = solve_ms
    roof["flops_per_launch"] = flops
    roof["unit_of_work"] = "vector-iteration"
    roof["units_per_launch"] = float(it_all.sum())
    if engine == "mfma":
        # Table I's count of the paper's primal steps (residual check, F
        # half-step, V residual, V aggregation over the users' VRs), which this
        # engine does not execute: it iterates in the dual space on the Gram
        # matrix (formed by the refresh), so achieved/peak on this count is
        # no utilisation figure and can exceed 1
        roof["count"] = "executed dual-space flops: Gram products over the overlap sets + x = H^H q + fresh residual"
        roof["primal_table_i_flops_per_launch"] = flops_primal
        roof["primal_table_i_over_peak"] = flops_primal / (solve_ms * 1e-3) / PEAK_MFMA_F32

    out = {
        "metric": METRIC, "value": value, "unit": "vectors/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if c128 else "f32", "data": "synthetic",
        "timing": "eager launches" if args.eager else
                  "HIP graph of the step (refresh + forward solve + adjoint), replayed (eager: %.4f ms per step)"
                  % ms_eager,
        "config": {"workload": WORKLOADS[wl], "variant": args.variant, "engine": engine,
                   "tile_waves": int(eng[2]), "tile_waves_adjoint": int(eng[9]), "persistent": int(eng[4]),
                   "wave_owned_tile_waves": int(eng[10]), "wave_owned_blocks_per_wave": int(eng[11]),
                   "entries_per_thread": int(eng[6]), "drops": len(drops), "vectors": B, "tol": tol,
                   "step": "vrk_plan_refresh (row norms, channel and Gram tiles) + vrk_solve + vrk_solve_adjoint"},
        "orthogonal_set_mean": float(np.mean([len(plan.query(j, vrk.Q_FSET)) for j in range(len(drops))])),
        "roofline": roof,
        "bind_ms": bind_ms,
        "accuracy": {"max_rel_err": worst, "mean_rel_err": errsum / B,
                     "all_converged": bool(np.all(fl_all == 1)), "mean_iters": float(it_all.mean()),
                     "max_iters": int(it_all.max()),
                     "adjoint_mean_iters": float(stats_adj[0].float().mean().item()),
                     "adjoint_max_iters": int(stats_adj[0].max().item()),
                     "adjoint_all_converged": bool((stats_adj[2] == 1).all().item())},
    }
    if ms_reuse is not None:
        out["channel_reused"] = {"ms_per_step": ms_reuse, "vectors_per_s": B / (ms_reuse * 1e-3),
                                 "note": "forward solve + adjoint only, the channel's tiles kept from the "
                                         "previous step (many symbol batches per channel)"}
    if tuned_ms is not None:
        out["config"]["autotuned_ms"] = tuned_ms
    if args.p_vis is not None:
        out["config"]["p_vis"] = args.p_vis   # overrides the 0.35 in the workload text

    # per-variant forward rates on the same batch and engine choice
    if not args.no_variants and wl == "many_rhs":
        rates = {}
        # the four variants with the default rule, then the benchmark rules of
        # the single-row sweep: greedy Kaczmarz (max), energy and uniform RK
        for name, var, rule in (("grk", "grk", "baiwu"), ("ahk", "ahk", "baiwu"), ("vr_ogrk", "vr_ogrk", "baiwu"),
                                ("vr_oahk", "vr_oahk", "baiwu"), ("gk_max", "grk", "max"),
                                ("rk_energy", "grk", "energy"), ("urk_uniform", "grk", "uniform")):
            sv_specs = [vrk.ProblemSpec(sp.H, d.vr_start, d.vr_len, d.xi, sp.S, torch.zeros_like(sp.X),
                                        torch.zeros_like(sp.V)) for sp, d in zip(specs, drops)]
            o = vrk.options(variant=var, select=rule, dtype=dname, engine=engine_opt, tol=tol,
                            tile_waves=args.tile_waves, persistent=args.persistent)
            pv = vrk.Plan(sv_specs, o)
            sv = pv.stats_buffers()
            pv.solve(stream=stream, stats=sv)
            torch.cuda.synchronize()
            reps = 3 if var in ("grk", "vr_ogrk") else 10
            reps = 1 if rule in ("energy", "uniform") else reps
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                pv.solve(stream=stream, stats=sv)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            Xr, _ = oracle.rzf(drops[0].H, drops[0].vr_start, drops[0].vr_len, drops[0].S, drops[0].xi)
            e2 = np.linalg.norm(sv_specs[0].X.cpu().numpy() - Xr, axis=1) / np.linalg.norm(Xr, axis=1)
            rates[name] = {"variant": var, "select": rule, "vectors_per_s": B / (ms * 1e-3), "ms": ms,
                           "max_rel_err": float(e2.max()), "mean_iters": float(sv[0].float().mean().item())}
            del pv
        out["variants_fwd"] = rates

    # plain single-instance solver: one vector per launch (vector engine), fwd + adjoint
    if not args.no_plain:
        d0, sp0 = drops[0], specs[0]
        n_plain = min(32, d0.nrhs)
        rate, us, Xl = plain_leg(d0, sp0, cdt, args.variant, tol, n_plain, stream)
        i = n_plain - 1
        Xr1, _ = oracle.rzf(d0.H, d0.vr_start, d0.vr_len, d0.S[i:i + 1], d0.xi, masks=d0.vr_mask,
                            n_sub=d0.n_sub)
        e1 = float(np.linalg.norm(Xl.cpu().numpy()[0] - Xr1[0]) / np.linalg.norm(Xr1[0]))
        out["plain"] = {"vectors_per_s": rate, "us_per_vector": us,
                        "engine": "vector, one vector per launch, fwd+adjoint, %d launches in a HIP graph" % n_plain,
                        "sample": n_plain, "rel_err_last": e1}
        out["speedup_vs_plain"] = value / rate
        out["plain_c1"] = plain_c1(stream)

    # FP64 oracle on the host: the same work (forward iterations with the same
    # variant and tolerance, plus the closed-form gradient) on a bounded
    # sample, and the legs of the CPU baseline plan
    if not args.no_cpu_baseline:
        thr = oracle.num_threads()
        step_cpu, legs = cpu_baseline(drops, args.variant, tol, wl, thr)
        out["cpu_baseline"] = {"value": step_cpu[0], "unit": "vectors/s", "cores": thr, "kind": "oracle",
                               "sample": step_cpu[1], "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                               "legs": legs}
    if args.copy_mb:
        src = torch.ones(args.copy_mb * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = args.copy_mb * 1048576
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
