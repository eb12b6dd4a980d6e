#!/usr/bin/env python3
"""Benchmark of the batched Step-LISTA forward + backward on one MI355X.

One step = one call of the whole hot path over the batch: correlations
c = D^T x, T fused layers forward, the objective, the backward seed, T fused
layers back and the reductions that give d(mean F)/d alpha. Inputs are
resident in HBM before timing starts. Throughput is sample-layers per
second (N * T per step). Both precisions of the contraction are timed (BF16
operands on MFMA, and FP32); `value` is the BF16 figure, and the FP32 one and
the objective gaps of both are reported beside it.

Prints ONE JSON line. Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
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

METRIC = "sample-layers/s fwd+bwd (BF16-MFMA vs FP32) at fixed obj-gap; % MFMA/HBM peak"
PEAK = {"bf16_tflops": 2500.0, "fp32_tflops": 157.3, "hbm_gbs": 8000.0}


def launch_work(kind: str, N: int, m: int, T: int):
    """Algorithmic flops and HBM bytes of one launch of a persistent kernel.

    Units: one contraction of one sample costs 2 m^2 flops (P = Z G). The
    iterate and c = D^T x of a tile stay on chip across the layers, so a
    sample's algorithmic HBM traffic is c read once (4 m bytes) plus what the
    launch must store or read: each kept iterate of the tape is 4 m bytes.
      forward launch (all T layers + the final contraction for F and the
        seed): T contractions (layer 0 has none since z^0 = 0, the final one
        is G z^T); bytes 4 m N (T + 3): c once, T kept iterates, the copy of
        z^T and the seed v^{T-1}.
      backward launch (all T layers): T - 1 contractions; bytes 4 m N (T + 1):
        the seed, z^T, and z^t for 1 <= t < T.
    Both are m / 2 flop per byte: above the BF16 ridge (2.5 PFLOP/s over
    8 TB/s = 312) for m = 1024, so their roofline is the MFMA peak. Bytes
    the kernels move beyond these (the forward re-reads its rows of c every
    layer) are excess, visible in the measured traffic."""
    if kind == "forward_layer":
        return 2.0 * N * m * m * T, 4.0 * m * N * (T + 3)
    if kind == "backward_layer":
        return 2.0 * N * m * m * (T - 1), 4.0 * m * N * (T + 1)
    raise ValueError(kind)


# HBM traffic per launch on prec_256x1024 (ckpt_every = 1, tile variant 4) from
# rocprofv3 counters: FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB per dispatch; the
# factors make a plain 1 GiB device copy read 1 GiB and write 1 GiB). Valid only
# for the kernel sources they were taken on (sha256 below) and that variant.
MEASURED_TRAFFIC = {
    "sources_sha256": "1a9e08e245b647ac1515dfb141b495a5d987f105a82485efb3cc8e687853e0ef",
    "workload": "prec_256x1024",
    "variant": 4,
    "bytes": {
        ("bf16", "forward_layer"): (8593231.1875 * 2 + 13632287.3125) * 1024,
        ("bf16", "backward_layer"): (8315042.3125 * 2 + 9811.59375) * 1024,
        ("fp32", "forward_layer"): (13239599.9375 * 2 + 13632346.5625) * 1024,
        ("fp32", "backward_layer"): (13107342.4375 * 2 + 3201.65625) * 1024,
    },
}

KERNEL_SOURCES = ["common.hpp", "persist.hpp", "persist_body.hpp", "kernels_persist.hip",
                  "kernels_persist_bf16.hip", "kernels_persist_f32.hip"]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1905_11071_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, ckpt: int, variant: int, prec: str, kind: str):
    if (workload != MEASURED_TRAFFIC["workload"] or ckpt != 1 or variant != MEASURED_TRAFFIC["variant"]
            or kernel_sources_sha256() != MEASURED_TRAFFIC["sources_sha256"]):
        return None
    return MEASURED_TRAFFIC["bytes"].get((prec, kind))


def roofline(kind: str, avg_ms: float, N: int, m: int, T: int, prec: str, traffic=None) -> dict:
    flops, bytes_ = launch_work(kind, N, m, T)
    peak_f = PEAK["bf16_tflops"] if prec == "bf16" else PEAK["fp32_tflops"]
    ridge = peak_f * 1e12 / (PEAK["hbm_gbs"] * 1e9)
    sec = avg_ms * 1e-3
    tflops = flops / sec / 1e12
    gbs = bytes_ / sec / 1e9
    out = {"kernel": kind, "avg_ms": round(avg_ms, 4), "flops_per_launch": flops, "bytes_per_launch": bytes_,
           "mfma_frac": round(tflops / peak_f, 4), "hbm_frac": round(gbs / PEAK["hbm_gbs"], 4), "traffic": traffic}
    if traffic is not None:
        out["traffic_gbs"] = round(traffic / sec / 1e9, 1)
        out["traffic_over_algorithmic"] = round(traffic / bytes_, 3)
    if flops / bytes_ < ridge:
        out.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                    "frac": round(gbs / PEAK["hbm_gbs"], 4)})
    else:
        out.update({"bound": "mfma", "achieved": round(tflops, 2), "peak": peak_f, "unit": "TFLOP/s",
                    "frac": round(tflops / peak_f, 4)})
    return out


def time_precision(sl, torch, d, X, lam, alpha, prec, steps, warmup, ckpt):
    N, T = X.shape[0], alpha.shape[0]
    ws = d.workspace(N, T, prec, ckpt)
    for _ in range(warmup):
        sl.forward_backward(d, X, lam, alpha, prec=prec, ckpt_every=ckpt, ws=ws)
    torch.cuda.synchronize()
    sl.profile_begin()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    out = None
    for _ in range(steps):
        out = sl.forward_backward(d, X, lam, alpha, prec=prec, ckpt_every=ckpt, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sl.profile_end()
    ms = e0.elapsed_time(e1) / steps
    kernels = {k: v for k, v in prof.items() if k != "dropped" and v[0] > 0}
    dom = max((k for k in kernels if k in ("forward_layer", "backward_layer")), key=lambda k: kernels[k][1])
    Z, F, loss, dalpha, _ = out
    del ws
    return {"ms_per_step": ms, "wall_ms_per_step": wall * 1e3 / steps, "kernels": kernels, "dominant": dom,
            "Z": Z, "loss": float(loss.item()), "dalpha_norm": float(dalpha.norm().item())}


def gap_report(sl, torch, d, X, lam, alpha, Z_by_prec, n_sub=4096, T_ref=3000):
    """Objective gap of each precision's z^(T) on a sample subset, against a
    long FP32 ISTA run (T_ref layers, alpha = 1/L), all F evaluated the same
    way (slista_objective: FP32 residual, FP64 sums)."""
    sub = X[:n_sub].contiguous()
    a_ref = torch.full((T_ref,), float(alpha[0].item()), device=X.device, dtype=torch.float32)
    Zr, _, _, _ = sl.forward(d, sub, lam, a_ref, prec="fp32", want_f=False, want_loss=False, ckpt_every=0)
    fr = sl.objective(d, sub, lam, Zr).double().mean().item()
    out = {"reference": f"FP32 ISTA, {T_ref} layers, first {n_sub} samples; F by slista_objective"}
    for p, Z in Z_by_prec.items():
        out[f"gap_{p}"] = sl.objective(d, sub, lam, Z[:n_sub].contiguous()).double().mean().item() - fr
    if "bf16" in Z_by_prec and "fp32" in Z_by_prec:
        out["bf16_vs_fp32_rel"] = abs(out["gap_bf16"] - out["gap_fp32"]) / abs(out["gap_fp32"])
        out["within_2e-2"] = out["bf16_vs_fp32_rel"] <= 2e-2
    return out


def cpu_baseline(pb, alpha_np, n_sub: int) -> dict:
    """The FP64 oracle (numpy/OpenBLAS, untuned) on the first n_sub samples."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    Xs = pb.X[:n_sub]
    t0 = time.perf_counter()
    oracle.forward_backward(pb.D, Xs, pb.lam, alpha_np, dF=np.full(n_sub, 1.0 / n_sub))
    sec = time.perf_counter() - t0
    T = len(alpha_np)
    return {"value": round(n_sub * T / sec, 1), "unit": "sample-layers/s", "cores": int(threads),
            "kind": "oracle", "sample": f"first {n_sub} of {pb.N} samples, all {T} layers, fwd+bwd, FP64 "
                                        f"({sec:.1f} s)"}


def uneven_inputs(sl, torch, T: int):
    """The 64 problems of the uneven batch on the device: (dictionary, X, lambda,
    alpha) with alpha_t = (1/L)(1 + 0.3 U[0,1)), L from the library's power
    iteration (setup, not timed)."""
    import synth
    specs = synth.uneven_problem_specs(P=synth.UNEVEN["P"], seed=synth.UNEVEN["seed"])
    dev = torch.device("cuda:0")
    t0 = time.time()
    inputs = []
    for sp in specs:
        pb = synth.make_problem(sp["n"], sp["m"], sp["N"], sp["p"], sp["sigma"], sp["lam_frac"], sp["seed"])
        d = sl.Dictionary(torch.tensor(pb.D32(), device=dev))
        L, _ = d.lipschitz(max_iter=20_000, rtol=1e-7)
        alpha = torch.tensor(synth.perturbed_steps(L, T, seed=sp["seed"]), device=dev, dtype=torch.float32)
        inputs.append((d, torch.tensor(pb.X32(), device=dev), pb.lam, alpha))
    print(f"[bench] uneven batch: {len(specs)} problems set up in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    return specs, inputs


UNEVEN_TAIL = 40  # FP32 layers at the end of the BF16 schedule of the uneven batch


def uneven_report(sl, torch, specs, inputs, prec: str, T: int, ckpt: int, reps: int) -> dict:
    """Uneven multi-problem batch: 64 independent Lasso problems (n in [32, 512],
    m = 4n, N in [128, 8192]), forward + backward with checkpoints every `ckpt`
    layers, tiles autotuned per column-pass bucket, timed as replays of one
    captured HIP graph. prec: "fp32", "bf16", or "bf16+tail" (BF16 layers and
    FP32 contractions in the last UNEVEN_TAIL layers: the schedule that meets
    the 2e-2 objective-gap bar on these converged problems, where BF16 in every
    layer misses it; tests/test_gpu_uneven_full.py holds both to the oracle)."""
    import numpy as np
    dev = torch.device("cuda:0")
    lib_prec = sl.bf16_fp32_tail(UNEVEN_TAIL) if prec == "bf16+tail" else prec
    b = sl.Batch(inputs, prec=lib_prec, ckpt_every=ckpt)
    b.run()
    torch.cuda.synchronize()
    tuned = b.autotune()
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.replay()
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    Ns = np.array([sp["N"] for sp in specs], np.float64)
    ms_ = np.array([sp["m"] for sp in specs], np.float64)
    # useful contractions per sample: T forward (T-1 layers + the final G z^T) and T-1 backward
    flops = float(np.sum(2.0 * Ns * ms_ ** 2) * (2 * T - 1))
    # executed: the backward recomputes the interior of every segment but the last
    nseg = -(-T // ckpt)
    recomputed = (nseg - 1) * (ckpt - 1) if ckpt > 1 else 0
    executed = float(np.sum(2.0 * Ns * ms_ ** 2) * (2 * T - 1 + recomputed))
    if prec == "bf16+tail":
        # useful time at the peaks of the two precisions, by layer share
        f_tail = UNEVEN_TAIL / T
        peak = 1.0 / ((1 - f_tail) / 2.5e15 + f_tail / 157.3e12)
    else:
        peak = 2.5e15 if prec == "bf16" else 157.3e12
    out = {"workload": "uneven_64", "problems": len(specs), "T": T, "ckpt_every": ckpt, "prec": prec,
           "total_samples": int(Ns.sum()), "ms_per_step": round(ms, 3),
           "value": round(float(Ns.sum()) * T / (ms * 1e-3), 1), "unit": "sample-layers/s",
           "mfma_tflops": round(flops / (ms * 1e-3) / 1e12, 2), "mfma_frac": round(flops / (ms * 1e-3) / peak, 4),
           "executed_tflops": round(executed / (ms * 1e-3) / 1e12, 2),
           "executed_over_useful": round(executed / flops, 3),
           "tuned_variant_by_column_passes": tuned, "timing": "HIP graph replay"}
    if prec == "bf16+tail":
        out["schedule"] = f"BF16 layers 0..{T - UNEVEN_TAIL - 1}, FP32 layers {T - UNEVEN_TAIL}..{T - 1}"
        out["peak_note"] = "mfma_frac against the layer-share-weighted peak of BF16 and FP32"
    if prec == "bf16":
        out["objective_gap_note"] = ("misses the 2e-2 objective-gap bar on these converged problems (an expected "
                                     "failure in tests/test_gpu_uneven_full.py); not an equal-accuracy figure")
    b.close()
    return out


def training_report(sl, torch, iters: int) -> dict:
    """Step-size training (full-batch sub-gradient descent with backtracking)
    on the 64 x 256 learned-step workload (N = 4096, T = 20), FP32 and BF16:
    accepted iterations, final loss and wall time per accepted iteration."""
    import numpy as np
    import synth
    c = synth.CONFIGS["grad_64x256"]
    pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
    dev = torch.device("cuda:0")
    d = sl.Dictionary(torch.tensor(pb.D32(), device=dev))
    X = torch.tensor(pb.X32(), device=dev)
    L, _ = d.lipschitz(max_iter=100_000, rtol=1e-12)
    out = {"workload": "grad_64x256", "n": pb.n, "m": pb.m, "N": pb.N, "T": c["T"], "iterations": iters}
    for p in ("fp32", "bf16"):
        alpha = torch.full((c["T"],), float(np.float32(1.0 / L)), device=dev, dtype=torch.float32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses, eta = sl.train(d, X, pb.lam, alpha, iters, 1.0 / L, prec=p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc = len(losses) - 1
        out[p] = {"accepted": acc, "loss_start": losses[0], "loss_end": losses[-1],
                  "ms_per_accepted_iteration": round(dt * 1e3 / max(acc, 1), 3),
                  "alpha_L_first_last": [round(float(alpha[0]) * L, 3), round(float(alpha[-1]) * L, 3)]}
    d.close()
    return out


def baselines_report(sl, torch, reps: int) -> dict:
    """FISTA and Oracle-ISTA (the paper's comparison methods, per-layer
    kernels) on the 64 x 256 batched-forward workload (N = 10000, T = 40):
    sample-layers/s of the forward pass per precision. FISTA's useful work is
    2 m^2 flops per sample-layer (G y^t); Oracle-ISTA adds per sample and layer
    the power iteration for L_S on the support."""
    import numpy as np
    import synth
    c = synth.CONFIGS["fwd_64x256"]
    pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
    dev = torch.device("cuda:0")
    d = sl.Dictionary(torch.tensor(pb.D32(), device=dev))
    X = torch.tensor(pb.X32(), device=dev)
    L, _ = d.lipschitz(max_iter=100_000, rtol=1e-12)
    N, T, m = pb.N, c["T"], pb.m
    alpha = torch.full((T,), float(np.float32(1.0 / L)), device=dev, dtype=torch.float32)
    out = {"workload": "fwd_64x256", "n": pb.n, "m": m, "N": N, "T": T, "pass": "forward"}
    runs = {"fista": lambda p: sl.fista(d, X, pb.lam, alpha, prec=p),
            "oista": lambda p: sl.oista(d, X, pb.lam, L, T, prec=p)}
    for name, fn in runs.items():
        out[name] = {}
        for p in ("fp32", "bf16"):
            fn(p)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                res = fn(p)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            r = {"ms_per_call": round(ms, 4), "value": round(N * T / (ms * 1e-3), 1), "unit": "sample-layers/s",
                 "loss": float(res[2].item())}
            if name == "fista":
                r["useful_tflops"] = round(2.0 * m * m * N * T / (ms * 1e-3) / 1e12, 2)
            out[name][p] = r
    d.close()
    return out


def ista_f64_report(sl, torch, reps: int) -> dict:
    """The double-precision ISTA workload ista_10x20 (n = 10, m = 20,
    N = 1000, T = 100, alpha = 1/L, the objective at every layer):
    slista_forward_f64, FP64 throughout, timed with HIP events over `reps`
    calls after a warm-up. Work per sample-layer in the factored form the
    FP64 path uses: 4 n m flops (D z, then D^T r; zero coordinates of z are
    skipped, so fewer are executed). A call is one wave per sample through
    100 dependent layers: latency bounds it, not a peak."""
    import synth
    c = synth.CONFIGS["ista_10x20"]
    pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
    dev = torch.device("cuda:0")
    d = sl.Dictionary(torch.tensor(pb.D32(), device=dev))
    L, _ = d.lipschitz(max_iter=100_000, rtol=1e-12)
    N, T = pb.N, c["T"]
    X = torch.tensor(pb.X, device=dev, dtype=torch.float64)
    alpha = torch.full((T,), 1.0 / L, device=dev, dtype=torch.float64)
    call = lambda: sl.forward_f64(d, X, pb.lam, alpha, f_trace=True)  # noqa: E731
    for _ in range(3):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 4.0 * pb.n * pb.m * N * T
    res = {"workload": "ista_10x20", "n": pb.n, "m": pb.m, "N": N, "T": T, "pass": "forward, F at every layer",
           "alpha": "1/L", "dtype": "f64", "ms_per_call": round(ms, 4), "value": round(N * T / (ms * 1e-3), 1),
           "unit": "sample-layers/s", "useful_gflops": round(flops / (ms * 1e-3) / 1e9, 2),
           "bound": "latency (one wave per sample, 100 dependent layers)", "loss": float(out[2].item())}
    d.close()
    return res


def configs_report(sl, torch, reps: int) -> dict:
    """The two 64 x 256 Gaussian workloads beside the headline one:
      fwd_64x256  batched ISTA forward, N = 10 000, T = 40, alpha = 1/L, no tape;
      grad_64x256 forward + backward, N = 4096, T = 20, alpha = 1/L, every
                  iterate kept (the learned-step workload).
    Each in FP32 (the workload's precision) and BF16, with the tile variant
    picked by slista_autotune for that workload (smaller tiles spread these
    few samples over more CUs), timed with HIP events over `reps` calls after
    a warm-up, with the library's per-kernel times from one more call. Useful flops: 2 m^2 per sample and contraction
    (forward T - 1 layers, plus the final G z^T where the objective or the
    seed is formed; backward T - 1 layers). At these sizes a call is tens to
    hundreds of microseconds: launch latency and the last wave of tiles
    (N / 64 tiles on 256 CUs) bound them, not the MFMA or HBM peaks, so the
    fractions below are low by construction."""
    import numpy as np
    import synth
    out = {}
    dev = torch.device("cuda:0")
    for wl, fb in (("fwd_64x256", False), ("grad_64x256", True)):
        c = synth.CONFIGS[wl]
        pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
        d = sl.Dictionary(torch.tensor(pb.D32(), device=dev))
        X = torch.tensor(pb.X32(), device=dev)
        L, _ = d.lipschitz(max_iter=100_000, rtol=1e-12)
        N, T, m = pb.N, c["T"], pb.m
        alpha = torch.full((T,), float(np.float32(1.0 / L)), device=dev, dtype=torch.float32)
        ent = {"workload": wl, "n": pb.n, "m": m, "N": N, "T": T,
               "pass": "forward+backward" if fb else "forward", "alpha": "1/L"}
        flops = 2.0 * N * m * m * ((T - 1) + (T if fb else 0))
        for p in ("fp32", "bf16"):
            best, tune_ms = sl.autotune(d, X, pb.lam, alpha, prec=p, ckpt_every=1)
            ws = d.workspace(N, T, p, 1 if fb else 0)
            if fb:
                call = lambda: sl.forward_backward(d, X, pb.lam, alpha, prec=p, ckpt_every=1, ws=ws)  # noqa: E731
            else:
                call = lambda: sl.forward(d, X, pb.lam, alpha, prec=p, want_f=False, want_loss=False,  # noqa: E731
                                          ckpt_every=0, ws=ws)
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            sl.profile_begin()
            call()
            torch.cuda.synchronize()
            prof = sl.profile_end()
            peak = PEAK["bf16_tflops"] if p == "bf16" else PEAK["fp32_tflops"]
            tf = flops / (ms * 1e-3) / 1e12
            ent[p] = {"ms_per_call": round(ms, 4), "value": round(N * T / (ms * 1e-3), 1),
                      "unit": "sample-layers/s", "useful_tflops": round(tf, 2), "mfma_frac": round(tf / peak, 4),
                      "bound": "launch latency and tail (see docstring)", "tile_variant": int(best),
                      "kernels_ms": {k: [v[0], round(v[1], 4)] for k, v in prof.items() if k != "dropped" and v[0] > 0}}
            del ws
        out[wl] = ent
        d.close()
    return out


def lista_report(sl, torch, reps: int, precs) -> dict:
    """Coupled LISTA forward+backward (all parameter gradients, dW included) on
    the 64 x 256 Gaussian workload, N = 10000, T = 40: sample-layers/s and the
    useful contraction rate. Useful flops per call: forward 2 contractions of
    2nm per sample-layer, backward 3 (W v, D^T (W v), the sum for dW), plus
    the final residual and the seed: N (10 n m T + 4 n m)."""
    import synth
    c = synth.CONFIGS["lista_64x256"]
    pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
    dev = torch.device("cuda:0")
    d = sl.Dictionary(torch.tensor(pb.D32(), device=dev))
    L, _ = d.lipschitz(max_iter=100_000, rtol=1e-12)
    W, a, b = (torch.tensor(v, device=dev, dtype=torch.float32)
               for v in synth.lista_params(pb.D, L, c["T"], c["seed"], c["spread"]))
    X = torch.tensor(pb.X32(), device=dev)
    N, T, n, m = pb.N, c["T"], pb.n, pb.m
    flops = N * (10.0 * n * m * T + 4.0 * n * m)
    out = {"workload": "lista_64x256", "n": n, "m": m, "N": N, "T": T, "pass": "forward+backward (dW, dalpha, dbeta)"}
    for p in precs:
        ws = sl.lista_workspace(d, N, T, p, tape=True)
        for _ in range(2):
            sl.lista_forward_backward(d, X, pb.lam, W, a, b, prec=p, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            res = sl.lista_forward_backward(d, X, pb.lam, W, a, b, prec=p, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # per-class breakdown from one more call with per-launch events (which
        # add their own gaps, so it is not the timed figure)
        sl.profile_begin()
        sl.lista_forward_backward(d, X, pb.lam, W, a, b, prec=p, ws=ws)
        torch.cuda.synchronize()
        prof = sl.profile_end()
        peak = PEAK["bf16_tflops"] if p == "bf16" else PEAK["fp32_tflops"]
        tf = flops / (ms * 1e-3) / 1e12
        out[p] = {"ms_per_call": round(ms, 4), "value": round(N * T / (ms * 1e-3), 1), "unit": "sample-layers/s",
                  "useful_tflops": round(tf, 2), "mfma_frac": round(tf / peak, 5), "loss": float(res[2].item()),
                  "kernels_ms": {k: [v[0], round(v[1], 4)] for k, v in prof.items() if k != "dropped" and v[0] > 0}}
        del ws
    d.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="prec_256x1024")
    ap.add_argument("--precs", default="bf16,fp32")
    ap.add_argument("--ckpt-every", type=int, default=1)
    ap.add_argument("--variant", type=int, default=0,
                    help="tile variant of the persistent kernels (0 = autotune on the workload)")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gap", action="store_true")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven 64-problem batch")
    ap.add_argument("--no-train", action="store_true", help="skip the step-size training report")
    ap.add_argument("--train-iters", type=int, default=30)
    ap.add_argument("--no-lista", action="store_true", help="skip the coupled LISTA report")
    ap.add_argument("--no-baselines", action="store_true", help="skip the FISTA / Oracle-ISTA report")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 64x256 forward and learned-step lines and the FP64 10x20 ISTA line")
    ap.add_argument("--lista-reps", type=int, default=10)
    ap.add_argument("--uneven-precs", default="bf16+tail,bf16,fp32")
    ap.add_argument("--uneven-reps", type=int, default=3)
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path needs no collectives); --gpus {args.gpus} "
              f"is not supported", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calib:
        n = 1 << 28  # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_each_way": n * 4, "copies": args.steps}))
        return 0

    import synth
    import paper_1905_11071_amd as sl

    cfg = synth.CONFIGS[args.workload]
    print(f"[bench] generating {args.workload} {cfg}", file=sys.stderr, flush=True)
    pb = synth.make_problem(cfg["n"], cfg["m"], cfg["N"], cfg["p"], cfg["sigma"], cfg["lam_frac"], cfg["seed"])
    dev = torch.device("cuda:0")
    D = torch.tensor(pb.D32(), device=dev)
    X = torch.tensor(pb.X32(), device=dev)
    d = sl.Dictionary(D)
    sl.set_tile_variant(args.variant)
    L, iters = d.lipschitz(max_iter=200_000, rtol=1e-13)
    T = cfg["T"]
    alpha = torch.full((T,), float(np.float32(1.0 / L)), device=dev, dtype=torch.float32)
    print(f"[bench] L={L:.9f} ({iters} power iterations)", file=sys.stderr, flush=True)

    tuned = {}
    res = {}
    for p in args.precs.split(","):
        if args.variant == 0:
            best, ms = sl.autotune(d, X, pb.lam, alpha, prec=p, ckpt_every=args.ckpt_every)
            tuned[p] = {"variant": best, "ms_per_call_by_variant": [round(x, 3) for x in ms]}
            print(f"[bench] autotune {p}: variant {best}, ms by variant {tuned[p]['ms_per_call_by_variant']}",
                  file=sys.stderr, flush=True)
        r = time_precision(sl, torch, d, X, pb.lam, alpha, p, args.steps, args.warmup, args.ckpt_every)
        dk = r["dominant"]
        n_l, tot = r["kernels"][dk]
        variant = tuned[p]["variant"] if args.variant == 0 else args.variant
        r["variant"] = variant
        r["roofline"] = roofline(dk, tot / n_l, pb.N, pb.m, T, p,
                                 measured_traffic(args.workload, args.ckpt_every, variant, p, dk))
        r["value"] = pb.N * T / (r["ms_per_step"] * 1e-3)
        res[p] = r
        print(f"[bench] {p}: {r['ms_per_step']:.3f} ms/step, {r['value']:.4g} sample-layers/s, "
              f"kernels={ {k: (v[0], round(v[1], 3)) for k, v in r['kernels'].items()} }",
              file=sys.stderr, flush=True)

    gap = None
    if not args.no_gap:
        gap = gap_report(sl, torch, d, X, pb.lam, alpha, {p: r["Z"] for p, r in res.items()})
        print(f"[bench] gap {gap}", file=sys.stderr, flush=True)

    uneven = None
    if not args.no_uneven:
        ucfg = synth.UNEVEN
        uneven = {}
        specs, inputs = uneven_inputs(sl, torch, ucfg["T"])
        for p in args.uneven_precs.split(","):
            uneven[p] = uneven_report(sl, torch, specs, inputs, p, ucfg["T"], ucfg["ckpt_every"], args.uneven_reps)
            print(f"[bench] uneven {p}: {uneven[p]}", file=sys.stderr, flush=True)
        for dd, _, _, _ in inputs:
            dd.close()
        del inputs

    train = None
    if not args.no_train:
        train = training_report(sl, torch, args.train_iters)
        print(f"[bench] training {train}", file=sys.stderr, flush=True)

    lista = None
    if not args.no_lista:
        lista = lista_report(sl, torch, args.lista_reps, ("fp32", "bf16"))
        print(f"[bench] lista {lista}", file=sys.stderr, flush=True)

    configs = ista64 = None
    if not args.no_configs:
        configs = configs_report(sl, torch, 20)
        print(f"[bench] 64x256 workloads {configs}", file=sys.stderr, flush=True)
        ista64 = ista_f64_report(sl, torch, 20)
        print(f"[bench] ista_10x20 fp64 {ista64}", file=sys.stderr, flush=True)

    baselines = None
    if not args.no_baselines:
        baselines = baselines_report(sl, torch, 5)
        print(f"[bench] baselines {baselines}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pb, np.asarray(alpha.cpu().numpy(), np.float64), min(args.cpu_sample, pb.N))
        print(f"[bench] cpu baseline {cpu}", file=sys.stderr, flush=True)

    head = "bf16" if "bf16" in res else next(iter(res))
    h = res[head]
    line = {
        "metric": METRIC,
        "value": round(h["value"], 1),
        "unit": "sample-layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": pb.n, "m": pb.m, "N": pb.N, "T": T,
                   "pass": "forward+backward", "ckpt_every": args.ckpt_every, "alpha": "1/L",
                   "contraction": "BF16 MFMA, FP32 accumulate" if head == "bf16" else "FP32 MFMA"},
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "per_precision": {p: {"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                              "roofline": r["roofline"], "tile_variant": r["variant"],
                              "kernels_ms": {k: [v[0], round(v[1] / args.steps, 4)] for k, v in r["kernels"].items()},
                              "loss": r["loss"]}
                          for p, r in res.items()},
        "objective_gap": gap,
        "workloads_64x256": configs,
        "workload_ista_10x20": ista64,
        "uneven_batch": uneven,
        "training": train,
        "lista": lista,
        "fista_oista": baselines,
        "autotune": tuned or {"forced_variant": args.variant},
    }
    print(json.dumps(line))
    d.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
