#!/usr/bin/env python
"""Throughput of the GP-fit + EI-scoring hot path on one MI355X.

One step = one Bayesian-optimisation iteration of a sub-search: fit the
Gaussian-process surrogate (float64 Cholesky, inverse factor, alpha, log
marginal likelihood), score the candidate pool and return the next
configuration (the EI argmax, read back to the host), with the fit's status
checked.  Inputs are resident in HBM before the timed region.

Default workload (c4, the metric's "GP vs MLP-prescreen+GP"): d=20, 4096
evaluations, a 1,048,576-candidate pool; the prescreen arm (an MLP ensemble
trained on the evaluations narrows the pool, the exact GP judges the
survivors) is `value`, the plain GPU GP over the whole pool is reported
beside it with the top-1 agreement of the two over 10 replicates.  Other
workloads (--workload): c1, c2 / c2-s (d=20, n=512, 65536 candidates, float32
matrix cores), c3 (three batched launches of 64 sub-searches), c5 / c5-s
(d=40, n=2048, 262144 candidates).

Prints one JSON line with the throughput (candidates/s over whole steps), the
roofline of the dominant kernel (timed with HIP events on the stream it runs
on), the error against the float64 oracle, and the oracle's own throughput on
the host cores.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate EI scores/sec (GP vs MLP-prescreen+GP) at stated error vs FP64"
PEAKS = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}  # dense matrix-core TFLOP/s, MI355X

# HBM traffic of the scoring kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# runs of this benchmark, scaled by the same counters on a plain copy of known
# size.  Valid only while the kernel source is unchanged (hash below).
TRAFFIC = {
    "kernel_sha": "a93b750b83d89aa0",
    "workload": "c2",
    "fetch_kib": 5027.5,       # FETCH_SIZE per dispatch of k_score_fused
    "write_kib": 896.0,        # WRITE_SIZE per dispatch
    "fetch_scale": 262144 / 131086.5,  # 256 MiB copy: FETCH_SIZE reads half the bytes moved
    "write_scale": 1.0,
}
TRAFFIC["bytes_per_launch"] = round(1024 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"]
                                            + TRAFFIC["write_kib"] * TRAFFIC["write_scale"]))


def kernel_source_hash(files=("score.hip", "score_common.h", "gpbo_internal.h")):
    """Hash of the sources a kernel is built from (default: k_score_fused's)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2403_08131_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# The same counters for the network forward (k_mlp_fwd<false>) at c4: one
# launch over 1,048,576 candidates x 5 members.  Algorithmic bytes per launch:
# the float32 pool once (1,048,576 x 20 x 4) plus the member outputs
# (5 x 1,048,576 x 4) = 104.9 MB.
FWD_SOURCES = ("mlp.hip", "score_common.h")
FWD_TRAFFIC = {
    "kernel_sha": "53478e7cb7a4798f",
    "fetch_kib": 44014.5,
    "write_kib": 20480.0,
    "fetch_scale": 262144 / 131083.5,
    "write_scale": 1.0,
    # the same pass over the pool, full occupancy, counters per dispatch:
    # vector-ALU busy share (VALUBusy) and matrix-core busy share (MfmaUtil)
    "valu_busy_pct": 57.6,
    "mfma_util_pct": 18.6,
    "valu_insts_per_wave": 1650,
    "mfma_insts_per_wave": 144,
}
# the vector-ALU issue rate of the chip in lane instructions per second
# (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz)
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9 / 1e12
FWD_TRAFFIC["bytes_per_launch"] = round(1024 * (FWD_TRAFFIC["fetch_kib"] * FWD_TRAFFIC["fetch_scale"]
                                                + FWD_TRAFFIC["write_kib"] * FWD_TRAFFIC["write_scale"]))


# Above this many observations the library scores float32 pools on the
# chunked large-n path (mirrors the library's own threshold).
LARGE_N_MIN = 1024


def flops_per_candidate(n, d, path="fused"):
    """Algorithmic flops per candidate of the timed kernel.  Fused kernel:
    triangular variance n(n+1), distances in matrix form 2nd, mean 2n, sum of
    squares 2n.  Large-n path: its timed kernel is the triangular product
    with the sum-of-squares epilogue, n(n+1) + 2n."""
    if path == "large":
        return n * (n + 1) + 2 * n
    return n * (n + 1) + 2 * n * d + 4 * n


def workload(name):
    from paper_2403_08131_amd import inputs as I
    if name in ("c2", "c2-s"):
        return I.make_config(name), "fp32"
    if name in ("c5", "c5-s"):
        return I.make_config(name), "fp32"
    if name == "c1":
        return I.make_config("c1"), "fp64"
    raise SystemExit(f"unknown workload {name}")


def describe(p, prec):
    kern = "SE-ARD" if p.kernel == 0 else "Matern-5/2"
    return {"workload": f"{p.name}: d={p.d} n={p.n} m={p.m} {kern} {prec} contractions, fp64 fit",
            "d": p.d, "n": p.n, "m": p.m, "kernel": kern, "precision": prec,
            "lengthscale": "log-uniform [0.05,1]" + (" x sqrt(d)" if p.name.endswith("-s") else "")}


def cpu_baseline(p, budget_s=15.0):
    """The float64 oracle on the host cores: full fit, plus scoring a bounded
    sample of the same candidate pool; the rate is extrapolated to a whole
    step (fit + all m candidates)."""
    from oracle import oracle as O
    kind = O.SE if p.kernel == 0 else O.MATERN52
    t0 = time.perf_counter()
    f = O.fit(p.X, p.y, p.lengthscale, kind, p.signal_var, p.noise_var)
    t_fit = time.perf_counter() - t0
    probe = min(p.m, 256)
    t0 = time.perf_counter()
    O.score(f, p.Xc[:probe])
    t_probe = time.perf_counter() - t0
    per = t_probe / probe
    sample = int(min(p.m, max(probe, budget_s / max(per, 1e-9))))
    t0 = time.perf_counter()
    O.score(f, p.Xc[:sample])
    t_s = time.perf_counter() - t0
    per = t_s / sample
    step = t_fit + p.m * per
    return {"value": p.m / step, "unit": "candidates/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"fit n={p.n} ({t_fit:.3f} s) + scoring {sample} of {p.m} candidates "
                      f"({t_s:.2f} s); rate = m / (t_fit + m * t_per_candidate)"}


def error_vs_oracle(p, prec, ctx, model, Xc_dev, sample=512):
    import torch
    from oracle import oracle as O
    from paper_2403_08131_amd import gpbo as G
    kind = O.SE if p.kernel == 0 else O.MATERN52
    f = O.fit(p.X, p.y, p.lengthscale, kind, p.signal_var, p.noise_var)
    idx = np.linspace(0, p.m - 1, sample).astype(np.int64)
    ref = O.score(f, p.Xc[idx])
    out = G.score(ctx, model, Xc_dev, prec)
    mu = out["mu"].double().cpu().numpy()[idx]
    sg = out["sigma"].double().cpu().numpy()[idx]
    scale = f.ystd * math.sqrt(p.signal_var)
    e_mu = float(np.max(np.abs(mu - ref["mu"]) / np.maximum(np.abs(ref["mu"]), scale)))
    fl = ref["sigma"] ** 2 >= 1e-2 * scale ** 2
    e_sg = float(np.max(np.abs(sg - ref["sigma"])[fl] / ref["sigma"][fl])) if fl.any() else 0.0
    return {"e_mu": e_mu, "e_sigma": e_sg, "sampled_candidates": sample}


MLP_FWD_FLOPS = lambda D, H: 2 * (D * H + H * H + H)  # per sample per member


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    """Host cores this process may use (the GPU machine grants a share of its
    host; OMP_NUM_THREADS states it)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def c4_oracle_legs(p, ctx, model, Xc_dev, rescore_idx):
    """The float64 oracle on the c4 problem: its own throughput on the host
    cores (cpu_baseline: the exact method, fit plus scoring, on a bounded
    sample, one thread and all threads) and the error of the device's exact
    re-score stage against it (error_vs_fp64)."""
    from oracle import oracle as O
    from paper_2403_08131_amd import gpbo as G
    import torch
    t0 = time.perf_counter()
    f = O.fit(p.X, p.y, p.lengthscale, O.SE, p.signal_var, p.noise_var)
    t_fit = time.perf_counter() - t0
    nt = cpu_threads()
    n1, nall = 64, 64 * nt
    t0 = time.perf_counter()
    O.score(f, p.Xc[:n1], nthreads=1)
    t1 = (time.perf_counter() - t0) / n1
    t0 = time.perf_counter()
    O.score(f, p.Xc[n1:n1 + nall], nthreads=nt)
    tall = (time.perf_counter() - t0) / nall
    base = {"value": p.m / (t_fit + p.m * tall), "unit": "candidates/s", "cores": nt,
            "kind": "oracle", "cpu": cpu_model(),
            "single_thread": {"value": p.m / (t_fit + p.m * t1), "cores": 1},
            "sample": f"full-GP step of the exact method at d={p.d}, n={p.n}: the serial float64 "
                      f"fit timed whole ({t_fit:.1f} s), scoring timed on {n1} candidates with one "
                      f"thread ({t1 * 1e3:.2f} ms each) and {nall} with {nt} threads "
                      f"({tall * 1e3:.3f} ms each); rate = m / (t_fit + m * t_per_candidate)"}
    # error of the device's exact stage (the float32 large-n path at n=4096)
    # on 256 candidates spread over the pool, and the argmax over one
    # 4096-row re-score set (the rows the prescreen handed to the judge)
    idx = np.linspace(0, p.m - 1, 256).astype(np.int64)
    ref = O.score(f, p.Xc[idx], nthreads=nt)
    rows = G.gather_rows(ctx, torch.as_tensor(idx, device=Xc_dev.device), Xc_dev)
    out = G.score(ctx, model, rows, "fp32")
    mu = out["mu"].double().cpu().numpy()
    sg = out["sigma"].double().cpu().numpy()
    ei = out["ei"].double().cpu().numpy()
    scale = f.ystd * math.sqrt(p.signal_var)
    fl = ref["sigma"] ** 2 >= 1e-2 * scale ** 2
    err = {"e_mu": float(np.max(np.abs(mu - ref["mu"]) / np.maximum(np.abs(ref["mu"]), scale))),
           "e_sigma": float(np.max(np.abs(sg - ref["sigma"])[fl] / ref["sigma"][fl])) if fl.any() else 0.0,
           "abs_dEI_over_EImax": float(np.max(np.abs(ei - ref["ei"])) / max(ref["ei"].max(), 1e-300)),
           "sampled_candidates": 256}
    rs = np.sort(rescore_idx)
    ref_rs = O.score(f, p.Xc[rs], want=("ei",), nthreads=nt)["ei"]
    sub = G.gather_rows(ctx, torch.as_tensor(rs, device=Xc_dev.device), Xc_dev)
    got = G.score(ctx, model, sub, "fp32", want=("ei",), host_argmax=True)
    srt = np.sort(ref_rs)[::-1]
    best = int(np.argmax(ref_rs))
    err["rescore_set_argmax"] = ("identical" if got["argmax"] == best else
                                 "near-tie" if (srt[0] - srt[1] <= 1e-4 * srt[0] and
                                                ref_rs[got["argmax"]] >= srt[0] * (1 - 1e-4))
                                 else "different")
    err["rescore_set_rows"] = int(rs.size)
    return base, err


def run_c4(args):
    """Learned prescreen against the plain GPU GP (d=20, 4096 evaluations,
    1,048,576-candidate pool, one replicate per seed).

    Each step is one Bayesian-optimisation iteration that returns the next
    configuration.  Both arms fit the exact GP on the evaluations (float64
    Cholesky, queued without a synchronisation).
      full-GP arm:   score the whole pool on the float32 path, take the EI
                     argmax;
      prescreen arm: the trained network (5 members, trained once per
                     replicate on the model's own observations) ranks the
                     pool by its predicted mean (on a stream of its own,
                     concurrent with the fit), keeps the top K1; the exact
                     judge takes the K2 of them with the largest EI upper
                     bound (posterior mean and nearest-observation variance
                     bound), scores those exactly and returns the EI argmax,
                     certified when no other of the K1 can beat it.
    The timed steps cycle through the replicates.  `value` is the prescreen
    arm's pool candidates per second; the full-GP arm, top-1 agreement of
    the two arms per replicate, the training time and both arms' dominant
    kernels are reported beside it."""
    import torch
    from paper_2403_08131_amd import gpbo as G
    from paper_2403_08131_amd import inputs as I

    E, H, K1, K2 = 5, 256, args.k1, args.k2
    dev = torch.device("cuda", 0)
    # both arms' GP work on a created stream: work there neither waits for
    # nor holds up the network's stream (the legacy default stream would
    # serialise with it), and the fit's launch sequence replays from a graph
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    ctx = G.Context(0)
    # the network works on a stream of its own (default priority), so its
    # pass over the pool runs concurrently with the GP fit; the judge waits
    # for both
    s_net = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s_net):
        ctx_net = G.Context(0)
    reps = []
    for rep in range(args.replicates):
        p = I.make_config("c4", replicate=rep)
        r = dict(p=p, X=torch.tensor(p.X, device=dev), y=torch.tensor(p.y, device=dev),
                 Xc=torch.tensor(p.Xc, dtype=torch.float32, device=dev))
        model = G.fit(ctx, r["X"], r["y"], p.lengthscale, p.kernel, p.signal_var, p.noise_var)
        init = I.mlp_init(p.extra["init_rng"], E, p.d, H)
        # the network lives on the network's context (its stream)
        net = G.Mlp(ctx_net, G.Mlp.pack(**init, device=dev), E, p.d, H)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = net.train_on_model(model, steps=args.train_steps, lr=args.lr)
        torch.cuda.synchronize()
        r["train_ms"] = (time.perf_counter() - t0) * 1e3
        r["loss"] = float(hist[-1].mean().item())
        model.free()
        # the network's pass as a persistent grid of one workgroup per compute
        # unit (40 KB of LDS, 4 waves): every CU keeps room for one of the
        # fit's 78 KB tile workgroups, so the fit on the GP stream runs beside
        # the pass at nearly its own speed (measured at c4: 5.43 ms per step
        # against 5.55 with two workgroups per CU and 5.77-5.89 filling the GPU)
        net.set_occupancy(args.fwd_occupancy)
        r["net"] = net
        reps.append(r)
    R = len(reps)

    def full_step(r):
        p = r["p"]
        model = G.fit_async(ctx, r["X"], r["y"], p.lengthscale, p.kernel, p.signal_var, p.noise_var)
        out = G.score(ctx, model, r["Xc"], "fp32", want=(), host_argmax=True)
        model.status()
        model.free()
        return out["argmax"]

    def pre_step(r):
        p = r["p"]
        # queue order: the network's pass over the pool (one launch), then the
        # fit (its launch sequence keeps the host busy for ~2.5 ms at n =
        # 4096), then the selection of the top K1 (a dozen small launches that
        # only the judge, after the fit, waits for)
        with torch.cuda.stream(s_net):
            outs = r["net"].forward(r["Xc"])
        model = G.fit_async(ctx, r["X"], r["y"], p.lengthscale, p.kernel, p.signal_var, p.noise_var)
        # the judge's float32 operands right behind the fit, beside the selection
        G.score_prepare_batched(ctx, [model], "fp32")
        with torch.cuda.stream(s_net):
            idx, _ = G.ens_select(ctx_net, outs, G.SELECT_LCB, 0.0, K1)
        done = torch.cuda.Event()
        done.record(s_net)
        torch.cuda.current_stream().wait_event(done)
        idx.record_stream(torch.cuda.current_stream())
        nxt, _, cert = G.score_subset(ctx, model, r["Xc"], idx, K2)  # synchronises
        model.status()
        model.free()
        return nxt, cert

    def timed(fn, steps, warmup):
        for i in range(warmup):
            fn(reps[i % R])
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        res = []
        a.record()
        for i in range(steps):
            res.append(fn(reps[i % R]))
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps, res

    ctx_net.timing()
    ctx_net.enable_timing(True)
    pre_ms, pre_res = timed(pre_step, args.steps, args.warmup)
    ctx_net.enable_timing(False)
    fwd_launches, fwd_ms = ctx_net.timing()
    ctx.timing()
    ctx.enable_timing(True)
    full_steps = max(R, 1)
    full_ms, full_res = timed(full_step, full_steps, 1)
    ctx.enable_timing(False)
    gemm_launches, gemm_ms = ctx.timing()
    picks_pre = {}
    for i, (nxt, cert) in enumerate(pre_res):
        picks_pre.setdefault(i % R, []).append((nxt, cert))
    picks_full = {i % R: a for i, a in enumerate(full_res)}
    agree = [picks_pre[k][0][0] == picks_full[k] for k in range(R)]
    certified = [picks_pre[k][0][1] for k in range(R)]
    stable = all(len({x[0] for x in v}) == 1 for v in picks_pre.values())

    p0 = reps[0]["p"]
    fwd_avg = fwd_ms / max(fwd_launches, 1)
    fl_fwd = MLP_FWD_FLOPS(p0.d, H) * E * p0.m
    fwd_waves = -(-p0.m // 64) * E * 4  # 64-sample tiles x members x 4 waves
    ach_fwd = fl_fwd / (fwd_avg * 1e-3) / 1e12
    gemm_avg = gemm_ms / max(gemm_launches, 1)
    fl_gemm = flops_per_candidate(p0.n, p0.d, "large") * p0.m * full_steps / max(gemm_launches, 1)
    ach_gemm = fl_gemm / (gemm_avg * 1e-3) / 1e12
    train_ms = float(np.mean([r["train_ms"] for r in reps]))
    res = {
        "metric": METRIC,
        "value": p0.m / (pre_ms * 1e-3),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": pre_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"c4: learned prescreen vs plain GPU GP, d={p0.d}, n={p0.n} "
                               f"evaluations, pool m={p0.m}; 5 x MLP {p0.d}-256-256-1 (BF16 "
                               f"matrix cores, {args.train_steps} Adam steps) keeps the top {K1} by "
                               f"predicted mean, the exact GP judge (EI bound, then FP32 EI on the "
                               f"top {K2}; FP64 fit) picks the next configuration",
                   "d": p0.d, "n": p0.n, "m": p0.m, "k1": K1, "k2": K2,
                   "train_steps": args.train_steps, "lr": args.lr, "replicates": R,
                   "timed_steps_cycle_replicates": True},
        "arms": {
            "prescreen": {"ms_per_step": pre_ms, "cand_per_s": p0.m / (pre_ms * 1e-3),
                          "top1_agreement_with_full_gp": {"agree": int(sum(agree)), "of": R},
                          "certified_within_prescreen_set": {"yes": int(sum(certified)), "of": R},
                          "picks_stable_across_steps": stable},
            "full_gp": {"ms_per_step": full_ms, "cand_per_s": p0.m / (full_ms * 1e-3)},
        },
        "speedup_vs_full_gp_at_equal_top1": (full_ms / pre_ms) if all(agree) else None,
        "speedup_vs_full_gp": full_ms / pre_ms,
        "train_ms": train_ms,
        "speedup_including_training": full_ms / (pre_ms + train_ms),
        "training_pays_off_after_steps": train_ms / max(full_ms - pre_ms, 1e-9),
        "final_train_loss": [round(r["loss"], 4) for r in reps],
        "roofline": {"bound": "mfma", "achieved": ach_fwd, "peak": PEAKS["bf16"],
                     "unit": "TFLOP/s", "frac": ach_fwd / PEAKS["bf16"],
                     "traffic": (FWD_TRAFFIC["bytes_per_launch"]
                                 if kernel_source_hash(FWD_SOURCES) == FWD_TRAFFIC["kernel_sha"]
                                 else None),
                     "algorithmic_bytes_per_launch": p0.m * p0.d * 4 + E * p0.m * 4,
                     "counters": ({k: FWD_TRAFFIC[k] for k in ("valu_busy_pct", "mfma_util_pct",
                                                            "valu_insts_per_wave",
                                                            "mfma_insts_per_wave")}
                                  if kernel_source_hash(FWD_SOURCES) == FWD_TRAFFIC["kernel_sha"]
                                  else None),
                     "kernel": "k_mlp_fwd", "flops_per_launch": fl_fwd, "avg_launch_ms": fwd_avg,
                     "note": "prescreen arm's dominant kernel; its GELU epilogues on the vector "
                             "ALU, not the matrix cores, bound it; it runs as a persistent grid "
                             "of %d workgroup(s) per CU to leave room for the concurrent fit"
                             % args.fwd_occupancy},
        # the same launch against the vector-ALU issue rate that bounds it:
        # lane instructions (the counted VALU instructions per wave x 64 lanes
        # x the launch's waves) per second, against 256 CUs x 4 SIMDs x 16
        # lanes x 2.4 GHz = 39.3 T lane instructions/s (packed FP32 is not
        # generated: the library is built without it)
        "roofline_valu": ({"bound": "alu", "kernel": "k_mlp_fwd",
                           "achieved": FWD_TRAFFIC["valu_insts_per_wave"] * 64 * fwd_waves
                           / (fwd_avg * 1e-3) / 1e12,
                           "peak": VALU_LANE_PEAK, "unit": "T lane instructions/s",
                           "frac": FWD_TRAFFIC["valu_insts_per_wave"] * 64 * fwd_waves
                           / (fwd_avg * 1e-3) / 1e12 / VALU_LANE_PEAK,
                           "avg_launch_ms": fwd_avg}
                          if kernel_source_hash(FWD_SOURCES) == FWD_TRAFFIC["kernel_sha"]
                          else None),
        "roofline_full_gp": {"bound": "mfma", "achieved": ach_gemm, "peak": PEAKS["fp32"],
                             "unit": "TFLOP/s", "frac": ach_gemm / PEAKS["fp32"], "traffic": None,
                             "kernel": "k_trigemm", "flops_per_launch": fl_gemm,
                             "avg_launch_ms": gemm_avg},
    }
    if not args.no_cpu:
        r0 = reps[0]
        p = r0["p"]
        model = G.fit(ctx, r0["X"], r0["y"], p.lengthscale, p.kernel, p.signal_var, p.noise_var)
        with torch.cuda.stream(s_net):
            idx, _ = r0["net"].prescreen_lcb(r0["Xc"], 0.0, K1)
        torch.cuda.synchronize()
        bound = G.score_bound(ctx, model, G.gather_rows(ctx, idx, r0["Xc"]), want=("ei_ub",))["ei_ub"]
        top = G.topk(ctx, bound, K2)
        rescore = idx.cpu().numpy()[top.cpu().numpy()]
        res["cpu_baseline"], res["error_vs_fp64"] = c4_oracle_legs(p, ctx, model, r0["Xc"], rescore)
        res["error_vs_fp64"]["argmax_agreement_10_seeds"] = {
            "prescreen_vs_full_gp": int(sum(agree)), "of": R,
            "note": "the full-GP arm's whole-pool argmax is the reference; the oracle cannot score "
                    "the 1,048,576-row pool at n=4096 in the bench's time"}
        model.free()
    for r in reps:
        r["net"].free()
    ctx_net.close()
    ctx.close()
    print(json.dumps(res), flush=True)


def run_c3(args):
    """Batched independent sub-searches: three launches of 64 problems each
    (coupling lambda = 0, 0.1, 0.5, one per launch), d in {2..12}, n in
    [16, 400], 8192 candidates per problem.  One step fits all 192 problems
    (one batched float64 launch sequence, queued without synchronising;
    ``--c3-fit per-launch``: one per launch), scores the pools of each
    launch with one persistent BF16 matrix-core launch (replayed from its
    HIP graph: the batch shape repeats from step to step), then reads the
    3 x 64 argmaxes back and checks the fits' statuses (host work that runs
    beside the next step's fit; the last step's before the clock stops).  `value` = candidates scored per second of whole
    steps.  The scoring kernel's own time is taken in a second pass with
    kernel timing on (eager launches bracketed by HIP events)."""
    import ctypes as C
    import torch
    from paper_2403_08131_amd import gpbo as G
    from paper_2403_08131_amd import inputs as I

    prec = args.prec or "bf16"
    pr = G.PREC[prec]
    dev = torch.device("cuda", 0)
    # a created stream: the library replays its launch graphs only there
    # (the legacy default stream cannot be captured)
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    ctx = G.Context(0)
    batches = []
    # the argmax of every sub-search of the three launches in one device
    # array, read back with one copy per step
    am_all = torch.empty((3, 64), dtype=torch.int64, device=dev)
    for li, lam in enumerate((0.0, 0.1, 0.5)):
        probs = I.make_c3(lam=lam, replicate=0)
        assert len(probs) == am_all.shape[1]
        specs = [dict(X=torch.tensor(p.X, device=dev), y=torch.tensor(p.y, device=dev),
                      lengthscale=p.lengthscale, kernel=p.kernel, signal_var=p.signal_var,
                      noise_var=p.noise_var) for p in probs]
        Xcs = [torch.tensor(p.Xc, dtype=torch.float32, device=dev) for p in probs]
        eis = [torch.empty(p.m, dtype=torch.float32, device=dev) for p in probs]
        am = am_all[li]
        em = torch.empty(len(probs), dtype=torch.float64, device=dev)
        batches.append(dict(lam=lam, probs=probs, specs=specs, Xcs=Xcs, eis=eis, am=am, em=em,
                            batch=G.ProblemBatch(specs),
                            ms=(C.c_int64 * len(probs))(*[x.shape[0] for x in Xcs]),
                            xs=(C.c_void_p * len(probs))(*[x.data_ptr() for x in Xcs]),
                            ep=(C.c_void_p * len(probs))(*[e.data_ptr() for e in eis])))
    B = len(batches[0]["probs"])
    # the fit of all three launches' sub-searches as one batched call (one
    # float64 launch sequence over 3 x 64 problems fills the GPU better than
    # three of 64), or one call per launch
    merged = args.c3_fit == "merged"
    everything = G.ProblemBatch([s for bt in batches for s in bt["specs"]])

    def launch(bt, models, mus=None, sgs=None):
        hs = (C.c_void_p * B)(*[mo.h.value for mo in models])
        mp = (C.c_void_p * B)(*[t.data_ptr() for t in mus]) if mus else None
        sp = (C.c_void_p * B)(*[t.data_ptr() for t in sgs]) if sgs else None
        ctx.check(G.lib().gpbo_score_batched(ctx.h, B, hs, bt["ms"], bt["xs"], pr, mp, sp, bt["ep"],
                                             C.c_void_p(bt["am"].data_ptr()),
                                             C.c_void_p(bt["em"].data_ptr())))

    def fit(group):
        st, models, status, _ = G.fit_batched(ctx, group, sync=False)
        if st != G.OK:
            raise SystemExit(f"batched fit failed: {status}")
        return models

    def finish(groups, kept):
        # the fits' statuses (read from the pinned copies made behind each
        # fit) and the models freed (their buffers return in stream order)
        for models in groups:
            st, status, _ = G.status_batched(ctx, models)
            if st != G.OK:
                raise SystemExit(f"batched fit failed: {status}")
        for models in kept:
            for mo in models:
                mo.free()

    def step(keep=False, pending=None):
        # the fits and the three scoring launches are queued back to back;
        # the previous step's status check and frees (host work only) run
        # while this step's fit is on the GPU; one synchronisation reads the
        # argmaxes
        kept = []
        if merged:
            models = fit(everything)
            # the scoring operands of all 192 fresh models in one launch pair
            G.score_prepare_batched(ctx, models, prec)
            for i, bt in enumerate(batches):
                kept.append(models[i * B:(i + 1) * B])
                launch(bt, kept[-1])
            groups = [models]
        else:
            for bt in batches:
                kept.append(fit(bt["batch"]))
                launch(bt, kept[-1])
            groups = kept
        if pending is not None:
            finish(*pending)
        picks = am_all.cpu()  # the next configuration of every sub-search
        if keep:
            st, status, _ = G.status_batched(ctx, [mo for models in groups for mo in models])
            if st != G.OK:
                raise SystemExit(f"batched fit failed: {status}")
            return picks, kept
        return picks, (groups, kept)

    def run_steps(k):
        # every step's whole work (fit, scores, argmaxes, status check,
        # frees) is done by the time the last step returns
        pending = None
        for _ in range(k):
            _, pending = step(pending=pending)
        if pending is not None:
            finish(*pending)

    run_steps(args.warmup)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    run_steps(args.steps)
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / args.steps
    m_step = sum(p.m for bt in batches for p in bt["probs"])

    # the fits alone, synchronised, for the breakdown
    t0 = time.perf_counter()
    for _ in range(3):
        for group in ([everything] if merged else [bt["batch"] for bt in batches]):
            _, models, _, _ = G.fit_batched(ctx, group)
            for mo in models:
                mo.free()
    torch.cuda.synchronize()
    fit_ms = (time.perf_counter() - t0) / 3 * 1e3

    # the scoring kernel alone: eager launches bracketed by HIP events
    ctx.timing()
    ctx.enable_timing(True)
    _, kept = step(keep=True)
    for _ in range(args.steps):
        for bt, models in zip(batches, kept):
            launch(bt, models)
    launches, k_ms = ctx.timing()
    ctx.enable_timing(False)
    k_avg = k_ms / max(launches, 1)
    fl_launch = sum(flops_per_candidate(p.n, p.d) * p.m for bt in batches for p in bt["probs"]) / 3
    achieved = fl_launch / (k_avg * 1e-3) / 1e12

    # error of the batched kernels' own outputs against the float64 oracle:
    # every problem of the three launches, mu and sigma on 256 candidates
    # spread over each pool, EI and the argmax over the whole pool
    from oracle import oracle as O
    errs = {"e_mu": 0.0, "e_sigma": 0.0, "abs_dEI_over_EImax": 0.0, "argmax_identical": 0,
            "argmax_near_tie": 0, "of": 0, "escalated_to_fp64": 0,
            "sample": "all 3 x 64 problems; mu, sigma on 256 candidates per pool, EI and argmax "
                      "over the whole pool"}
    bound = 1e-4 if prec == "fp32" else 5e-2
    for bt, models in zip(batches, kept):
        mus = [torch.empty(p.m, dtype=torch.float32, device=dev) for p in bt["probs"]]
        sgs = [torch.empty(p.m, dtype=torch.float32, device=dev) for p in bt["probs"]]
        launch(bt, models, mus, sgs)
        torch.cuda.synchronize()
        am = bt["am"].cpu().numpy()
        for k, (p, mo) in enumerate(zip(bt["probs"], models)):
            f = O.fit(p.X, p.y, p.lengthscale, O.SE, p.signal_var, p.noise_var)
            ref_all = O.score(f, p.Xc, want=("ei",))["ei"]
            idx = np.linspace(0, p.m - 1, 256).astype(np.int64)
            ref = O.score(f, p.Xc[idx])
            mu = mus[k].double().cpu().numpy()[idx]
            sg = sgs[k].double().cpu().numpy()[idx]
            ei = bt["eis"][k].double().cpu().numpy()
            scale = f.ystd * math.sqrt(p.signal_var)
            errs["e_mu"] = max(errs["e_mu"], float(np.max(np.abs(mu - ref["mu"]) /
                                                           np.maximum(np.abs(ref["mu"]), scale))))
            fl = ref["sigma"] ** 2 >= 1e-2 * scale ** 2
            if fl.any():
                errs["e_sigma"] = max(errs["e_sigma"],
                                      float(np.max(np.abs(sg - ref["sigma"])[fl] / ref["sigma"][fl])))
            errs["abs_dEI_over_EImax"] = max(errs["abs_dEI_over_EImax"], float(
                np.max(np.abs(ei - ref_all)) / max(ref_all.max(), 1e-300)))
            errs["escalated_to_fp64"] += int(prec == "fp32" and mo.stats()["kinv"] > G.ESCALATE_KINV)
            srt = np.sort(ref_all)[::-1]
            errs["of"] += 1
            if am[k] == int(np.argmax(ref_all)):
                errs["argmax_identical"] += 1
            elif srt[0] - srt[1] <= bound * srt[0] and ref_all[am[k]] >= srt[0] * (1 - bound):
                errs["argmax_near_tie"] += 1
    for models in kept:
        for mo in models:
            mo.free()

    res = {
        "metric": METRIC,
        "value": m_step / (ms_step * 1e-3),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"c3: 3 batched launches (lambda 0, 0.1, 0.5) x {B} sub-searches, "
                               f"d in 2..12, n in 16..400, 8192 candidates each, SE-ARD "
                               f"log-uniform [0.05,1], {prec} contractions, fp64 fit",
                   "B": B, "launches_per_step": 3, "m_per_problem": 8192,
                   "fit": ("one batched call over the 3 x 64 sub-searches" if merged
                           else "one batched call per launch"),
                   "n_per_problem": [p.n for p in batches[0]["probs"]][:8] + ["..."],
                   "precision": prec},
        "breakdown_ms": {"fits_per_step": fit_ms, "timed_kernel_per_step": 3 * k_avg},
        "error_vs_fp64": errs,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAKS[prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAKS[prec], "traffic": None, "kernel": "k_score_batched",
                     "flops_per_launch": fl_launch, "avg_launch_ms": k_avg,
                     "note": "bf16: squared distances on the fp32 matrix cores, the variance on "
                             "the bf16 ones; latency per work item (lookup, staging, four "
                             "phases) bounds it at these small n and d (vector ALU ~39 %, "
                             "matrix cores ~16 % busy)"},
    }
    ctx.close()
    print(json.dumps(res), flush=True)


def run_bo(args):
    """The whole optimisation on the paper's synthetic family (Sec. III-C,
    Table I case ``--case``): the interdependence analysis plans the searches
    (Sec. IV-B to IV-D), then every strategy runs its searches to the budget
    (5 initial configurations, 10 evaluations per parameter) through the
    batched driver -- one batched scoring call and one batched rank-one
    update per iteration.  Strategies, as in the paper's Table III:
    independent (one search per group), merged (the planner's searches) and
    joint (all 20 parameters in one search).  The parameters a search does
    not tune stay at the baseline configuration; at the end each strategy's
    best values are combined into one configuration and F is evaluated there.
    The metric is search iterations per second (one iteration of one search:
    its pool scored, its argmax evaluated, its model updated)."""
    import torch
    from paper_2403_08131_amd import bo as BO
    from paper_2403_08131_amd import gpbo as G
    from paper_2403_08131_amd import inputs as I

    dev = torch.device("cuda", 0)
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    ctx = G.Context(0)
    case = args.case
    rng = np.random.default_rng(4000 + case)
    lo, hi = I.PAPER_BOUNDS
    x0 = I.f32r(rng.uniform(lo, hi, 20))
    sw = I.sensitivity_sweep(x0)
    S = G.sensitivity(I.paper_groups(x0, case), I.paper_groups(sw, case))
    owner = [j // 5 for j in range(20)]
    _, ps, nsearch = G.plan_searches(S, owner)
    plans = {
        "independent": [list(range(5 * g, 5 * g + 5)) for g in range(4)],
        "merged": [[j for j in range(20) if ps[j] == k] for k in range(nsearch)],
        "joint": [list(range(20))],
    }
    prec = args.prec or "fp32"

    def evaluate_for(dims_list):
        def ev(b, X):
            Xf = np.repeat(x0[None, :], X.shape[0], axis=0)
            Xf[:, dims_list[b]] = X
            return I.paper_objective(Xf, case)
        return ev

    out = {}
    total_iters, total_s = 0, 0.0
    for name, dims_list in plans.items():
        searches = [BO.Search(dims=dl, lo=np.full(len(dl), lo), hi=np.full(len(dl), hi),
                              lengthscale=np.full(len(dl), 25.0), noise_var=1e-4)
                     for dl in dims_list]
        ev = evaluate_for(dims_list)
        # warm-up with other pools: autotuned batched-scoring shapes, captured
        # launch graphs and allocator pools for this strategy's batch shapes
        BO.run(ctx, searches, ev, pool_size=args.pool, prec=prec, seed=1000 + case)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = BO.run(ctx, searches, ev, pool_size=args.pool, prec=prec, seed=case)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        iters = sum(len(r.picks) for r in res)
        steps = max(len(r.picks) for r in res)
        xc = x0.copy()
        for dl, r in zip(dims_list, res):
            xc[dl] = r.best[0]
        out[name] = {"searches": [len(dl) for dl in dims_list], "evaluations": sum(r.y.size for r in res),
                     "F_combined": float(I.paper_objective(xc[None, :], case)[0]),
                     "best_per_search": [round(r.best[1], 4) for r in res],
                     "wall_s": dt, "loop_steps": steps, "ms_per_loop_step": dt / steps * 1e3,
                     "search_iterations": iters}
        total_iters += iters
        total_s += dt
    # the merged plan again with a batched refit instead of the rank-one
    # update (same pools and picks up to rounding), and the oracle's loop of
    # its first search on the host
    dims_list = plans["merged"]
    searches = [BO.Search(dims=dl, lo=np.full(len(dl), lo), hi=np.full(len(dl), hi),
                          lengthscale=np.full(len(dl), 25.0), noise_var=1e-4) for dl in dims_list]
    ev = evaluate_for(dims_list)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rr = BO.run(ctx, searches, ev, pool_size=args.pool, prec=prec, seed=case, update="refit")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = max(len(r.picks) for r in rr)
    out["merged"]["refit_instead_of_update"] = {
        "wall_s": dt, "ms_per_loop_step": dt / steps * 1e3,
        "F_combined_same": bool(np.allclose([r.best[1] for r in rr],
                                            out["merged"]["best_per_search"], atol=1e-4))}
    cpu = None
    if not args.no_cpu:
        from oracle import bo as OBO
        from oracle import oracle as O
        s0 = searches[0]
        g = np.random.default_rng(7)
        X0 = g.uniform(lo, hi, size=(5, s0.d))
        ev0 = lambda x: float(ev(0, x[None, :])[0])
        pools = [g.uniform(lo, hi, size=(args.pool, s0.d)) for _ in range(10 * s0.d - 5)]
        t0 = time.perf_counter()
        OBO.search(ev0, X0, [ev0(x) for x in X0], pools, s0.lengthscale, O.SE, 1.0, 1e-4)
        tc = time.perf_counter() - t0
        cpu = {"value": len(pools) / tc, "unit": "search-iterations/s", "cores": cpu_threads(),
               "kind": "oracle", "cpu": cpu_model(),
               "sample": f"the oracle's loop (refit, float64 EI over {args.pool} candidates) of the "
                         f"first planned search, d={s0.d}, {len(pools)} iterations"}
    res = {
        "metric": "BO search iterations/s (batched EI scoring + rank-one update per iteration)",
        "value": total_iters / total_s, "unit": "search-iterations/s", "n_gpus": 1,
        "steps": sum(v["loop_steps"] for v in out.values()), "warmup": 1,
        "ms_per_step": total_s / sum(v["loop_steps"] for v in out.values()) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"bo: the paper's 20-parameter synthetic family, case {case}; "
                               f"independent / merged (planned) / joint searches, 5 initial "
                               f"configurations, 10 evaluations per parameter, pools of {args.pool} "
                               f"uniform candidates, {prec} scoring",
                   "case": case, "pool": args.pool, "planned_searches": plans["merged"]},
        "strategies": out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def run_hyper(args):
    """Hyperparameter fitting of one c3 batch (64 sub-searches, d in 2..12, n
    in 16..400, literal draws): every problem from 4 starts (log-uniform
    lengthscales in [0.05, 1], signal variance in [0.5, 2], noise variance in
    [1e-4, 1e-1]), 100 Adam steps up the LML gradient in log space, all 256
    runs in one batched fit and one gradient launch pair per step.  The
    metric is LML-gradient evaluations per second (one evaluation = one fit
    and one gradient of one run); the gradient kernels are timed on their own
    as well, and the oracle's gradient on the host for one problem."""
    import torch
    from paper_2403_08131_amd import gpbo as G
    from paper_2403_08131_amd import inputs as I

    dev = torch.device("cuda", 0)
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    ctx = G.Context(0)
    probs = I.make_c3(lam=0.1, m=16)
    B, S, steps = len(probs), 4, args.hyper_steps
    ldt = max(p.d for p in probs) + 2
    rng = np.random.default_rng(77)
    th0 = np.zeros((B, S, ldt))
    lo = np.zeros((B, ldt))
    hi = np.zeros((B, ldt))
    for b, p in enumerate(probs):
        d = p.d
        th0[b, :, :d] = rng.uniform(np.log(0.05), 0.0, size=(S, d))
        th0[b, :, d] = np.log(rng.uniform(0.5, 2.0, size=S))
        th0[b, :, d + 1] = np.log(rng.uniform(1e-4, 1e-1, size=S))
        lo[b, :d + 2] = np.log([1e-3] * d + [1e-2, 1e-6])
        hi[b, :d + 2] = np.log([1e2] * d + [1e2, 1.0])
    dp = [dict(X=torch.tensor(p.X, device=dev), y=torch.tensor(p.y, device=dev)) for p in probs]
    # warm-up (graphs, allocator pools), then the timed fit
    G.fit_hyper_batched(ctx, dp, th0, lo, hi, steps=2, lr=0.05, want_models=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, status, th, lml, jit, _ = G.fit_hyper_batched(ctx, dp, th0, lo, hi, steps=steps, lr=0.05,
                                                      want_models=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = B * S * (steps + 1)
    # LML at the starting points (one start per problem) for the gain
    _, _, _, lml0, _, _ = G.fit_hyper_batched(ctx, dp, th0[:, :1, :], lo, hi, steps=0,
                                              want_models=False)
    # the gradient kernels alone on the 64 fitted models at the optimum
    pr = [dict(X=dp[b]["X"], y=dp[b]["y"], lengthscale=list(np.exp(th[b, :probs[b].d])),
               signal_var=float(np.exp(th[b, probs[b].d])),
               noise_var=float(np.exp(th[b, probs[b].d + 1]) + jit[b])) for b in range(B)]
    _, models, _, _ = G.fit_batched(ctx, pr)
    for _ in range(3):
        G.lml_grad_batched(ctx, models)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        G.lml_grad_batched(ctx, models)
    e1.record()
    torch.cuda.synchronize()
    g_ms = e0.elapsed_time(e1) / 20
    for m_ in models:
        m_.free()
    # algorithmic flops of one batched gradient: K^-1 from the inverse factor
    # (sum over tiles of 64^3 multiply-adds x (nb - I) slabs) ~ n^3 / 3 per model
    # as counted by the kernel, plus n^2 (d + 2) for the sums
    npads = [((p.n + 63) // 64) * 64 for p in probs]
    fl = sum(2 * np_ ** 3 / 3 + 2 * p.n * p.n * (p.d + 2) for np_, p in zip(npads, probs))
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        p = max(probs, key=lambda q: q.n)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 5.0:
            O.lml_grad(p.X, p.y, p.lengthscale, O.SE, 1.0, 1e-2)
            k += 1
        dt = (time.perf_counter() - t0) / k
        cpu = {"value": 1.0 / dt, "unit": "LML-gradient evaluations/s", "cores": 1,
               "kind": "oracle", "cpu": cpu_model(),
               "sample": f"the oracle's fit + LML gradient of the largest problem (n={p.n}, "
                         f"d={p.d}), serial, {k} evaluations"}
    res = {
        "metric": "LML-gradient evaluations/s (batched fit + gradient, multi-start Adam)",
        "value": evals / wall, "unit": "evaluations/s", "n_gpus": 1, "steps": steps,
        "warmup": 2, "ms_per_step": wall / (steps + 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp64", "data": "synthetic",
        "config": {"workload": f"hyper: one c3 batch (64 sub-searches, d 2..12, n 16..400), "
                               f"4 starts each, {steps} Adam steps (lr 0.05) in log space",
                   "problems": B, "starts": S},
        "lml_gain": {"mean_start_lml": float(np.mean(lml0)), "mean_final_lml": float(np.mean(lml)),
                     "problems_improved": int(np.sum(lml > lml0)), "of": B,
                     "jittered": int(np.sum(jit > 0))},
        "gradient_kernels": {"ms_per_batched_call": g_ms, "flops": fl,
                             "achieved_tflops": fl / (g_ms * 1e-3) / 1e12,
                             "peak_fp64_vector_tflops": PEAKS["fp64"],
                             "note": "float64 FMA on the vector ALU; latency-bound at these n"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--stream", default="default", choices=("created", "default"),
                    help="c1/c2/c5: torch's default stream (eager launches) or a created "
                         "stream (the fit's launch sequence replayed from a graph)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--path", default="auto", choices=("auto", "fused", "large"))
    ap.add_argument("--prec", default=None, choices=("fp32", "bf16"),
                    help="c3: precision of the score contractions (default bf16)")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--replicates", type=int, default=10)
    ap.add_argument("--k1", type=int, default=65536, help="c4: candidates the network keeps")
    ap.add_argument("--k2", type=int, default=4096, help="c4: candidates the judge scores exactly")
    ap.add_argument("--lr", type=float, default=3e-3, help="c4: Adam learning rate")
    ap.add_argument("--fwd-occupancy", type=int, default=1,
                    help="c4: network forward workgroups per compute unit (0 = fill the GPU)")
    ap.add_argument("--c3-fit", default="merged", choices=("merged", "per-launch"),
                    help="c3: fit the three launches' sub-searches in one batched call or one "
                         "call per launch")
    ap.add_argument("--hyper-steps", type=int, default=100, help="hyper: Adam steps per start")
    ap.add_argument("--case", type=int, default=3, help="bo: case of the paper's family (1..5)")
    ap.add_argument("--pool", type=int, default=65536, help="bo: candidates per search and iteration")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes three times "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        yb = torch.empty_like(x)
        for _ in range(3):
            yb.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the scoring path "
              "runs on one MI355X; see the sharding note in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "bo":
        return run_bo(args)
    if args.workload == "hyper":
        return run_hyper(args)

    import torch
    from paper_2403_08131_amd import gpbo as G

    p, prec = workload(args.workload)
    dev = torch.device("cuda", 0)
    # on a created stream the library replays the fit's launch sequence from
    # a graph per shape (the legacy default stream cannot be captured); the
    # whole step is host-bound at c2 and measures the same either way
    if args.stream == "created":
        torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    X = torch.tensor(p.X, device=dev)
    y = torch.tensor(p.y, device=dev)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xc = torch.tensor(p.Xc, dtype=dt, device=dev)
    ctx = G.Context(0)
    ctx.set_score_path(args.path)
    path = args.path
    if path == "auto":  # the library's own choice for these workloads
        path = "large" if prec == "fp32" and p.n > LARGE_N_MIN else "fused"

    def step():
        # fit and scoring queued back to back; one synchronisation (the argmax
        # read back), then the fit's status, which is already on the host side
        model = G.fit_async(ctx, X, y, p.lengthscale, p.kernel, p.signal_var, p.noise_var)
        out = G.score(ctx, model, Xc, prec)
        best = int(out["argmax"].item())  # the next configuration to evaluate
        model.status()  # raises if the factorisation failed
        model.free()
        return best

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    ctx.timing()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    launches, k_ms = ctx.timing()
    ctx.enable_timing(False)
    ms_step = ms_total / args.steps
    k_avg = k_ms / max(launches, 1)
    k_step = k_ms / args.steps  # timed-kernel time per step (one launch per chunk)

    # fit alone, for the breakdown
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        G.fit(ctx, X, y, p.lengthscale, p.kernel, p.signal_var, p.noise_var).free()
    fit_ms = (time.perf_counter() - t0) / 3 * 1e3

    fl = flops_per_candidate(p.n, p.d, path) * p.m  # per step
    achieved = fl / (k_step * 1e-3) / 1e12
    peak = PEAKS[prec]
    traffic = None
    if TRAFFIC.get("kernel_sha") == kernel_source_hash() and TRAFFIC.get("workload") == p.name:
        traffic = TRAFFIC["bytes_per_launch"]

    model = G.fit(ctx, X, y, p.lengthscale, p.kernel, p.signal_var, p.noise_var)
    err = error_vs_oracle(p, prec, ctx, model, Xc)
    model.free()

    res = {
        "metric": METRIC,
        "value": p.m / (ms_step * 1e-3),
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": describe(p, prec),
        "breakdown_ms": {"fit": fit_ms, "timed_kernel_per_step": k_step},
        "timed_kernel_launches_per_step": launches / args.steps,
        "timed_kernel_cand_per_s": p.m / (k_step * 1e-3),
        "error_vs_fp64": err,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": {"fused": "k_score_fused", "large": "k_trigemm"}[path],
                     "path": path, "flops_per_step": fl,
                     "flops_per_launch": fl * args.steps / max(launches, 1),
                     "avg_launch_ms": k_avg},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(p)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
