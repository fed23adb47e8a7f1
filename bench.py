#!/usr/bin/env python3
"""Throughput of the symmetric-contraction hot path on one MI355X.

Default workload: one single-site effective-Hamiltonian application
y = L . W . x . R (three U(1) pairwise contractions, Alg. "Single-site
Benchmark") at virtual bond dimension D = 4096 over charges -12..12, fp64.
A step is the whole application: for each of the three contractions the
operand permutes, the grouped sector GEMM with its fused output scatter and
the zero blocks.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  value = useful block flops (sum over coupled charges of
2 M N K) per second, whole job.  roofline = the grouped sector-GEMM kernel of
the two MFMA-bound contractions, timed with HIP events on its own stream
inside the timed region.  cpu_baseline = the CPU oracle (numpy blockwise,
fp64) timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                                     # GB/s
METRIC = "symmetric contract TFLOP/s (block flops) + % MFMA peak; max rel err vs FP64"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="heff_d4096", choices=["heff_d4096", "heff_d1024"])
    ap.add_argument("--precision", default="native", choices=["native", "f32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile configuration")
    ap.add_argument("--tune-cache", default=None, help="JSON file to read/write tuned tile configurations")
    return ap.parse_args()


def heff_workload(name):
    from paper_2508_10076_amd import synth
    if name == "heff_d4096":
        return synth.config3(), 3
    return synth.config2(), 2


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2508_10076_amd import synth, tk

    torch.cuda.set_device(0)
    cfg, cid = heff_workload(args.workload)
    ctx = tk.Context(0)
    stream = torch.cuda.Stream()

    # tensors and seeded inputs (identical draws to the parity tests)
    T = {}
    for i, k in enumerate(cfg["inputs"]):
        t = cfg["tensors"][k]
        T[k] = tk.tensor_create(ctx, t["sym"], t["cod"], t["dom"])
        T[k].storage[: T[k].nelem].copy_(torch.from_numpy(synth.normal(T[k].nelem, cid, i)))
    plans = []
    flops = 0.0
    for out, a, b, call in cfg["calls"]:
        T[out] = tk.tensor_create_contracted(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"],
                                             call["pAB"], call["qAB"])
        P = tk.Plan(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"], call["pAB"], call["qAB"],
                    T[out], precision=args.precision)
        info = P.info()
        flops += info["flops"]
        plans.append((P, T[a], T[b], T[out], info))
    torch.cuda.synchronize()

    # the MFMA-bound contractions: those whose GEMMs have K well above 16
    mfma_steps = [i for i, (P, *_r) in enumerate(plans) if P.gemms()[:, 2].max() > 64]
    gemm_flops = sum(plans[i][4]["flops"] for i in mfma_steps)

    # tile configuration per contraction, chosen by the autotuner
    from paper_2508_10076_amd import autotune
    tuning = {}
    for i in mfma_steps:
        P, A, B, Cc, _ = plans[i]
        if args.no_tune:
            break
        best, times = autotune.tune(P, lambda P=P, A=A, B=B, Cc=Cc: P.execute_stages(A, B, Cc, tk.STAGE_GEMM,
                                                                                       stream=stream),
                                    P.gemms().tolist(), stream, cache_path=args.tune_cache, force=True,
                                    tag=("f64", args.precision))
        tuning[f"step{i + 1}"] = {"tile": list(best), "ms": {"x".join(map(str, c)): round(t, 4)
                                                             for c, t in times.items()}}
    torch.cuda.synchronize()

    def step(ev=None):
        for i, (P, A, B, Cc, _) in enumerate(plans):
            if ev is not None and i in mfma_steps:
                P.execute_stages(A, B, Cc, tk.STAGE_PERMUTE, stream=stream)
                ev.append(torch.cuda.Event(enable_timing=True))
                ev[-1].record(stream)
                P.execute_stages(A, B, Cc, tk.STAGE_GEMM, stream=stream)
                ev.append(torch.cuda.Event(enable_timing=True))
                ev[-1].record(stream)
                P.execute_stages(A, B, Cc, tk.STAGE_ZERO, stream=stream)
            else:
                P.execute(A, B, Cc, stream=stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    evs = []
    t0.record(stream)
    for _ in range(args.steps):
        step(evs)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    ms_per_step = total_ms / args.steps
    gemm_ms = sum(evs[2 * j].elapsed_time(evs[2 * j + 1]) for j in range(len(evs) // 2))
    gemm_launches = len(evs) // 2
    gemm_avg_s = gemm_ms / 1e3 / gemm_launches
    achieved = gemm_flops / len(mfma_steps) / gemm_avg_s / 1e12
    value = flops * args.steps / (total_ms / 1e3) / 1e12
    peak_key = {"native": "f64", "f32": "f32", "bf16x3": "bf16"}[args.precision]

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "native" else args.precision,
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: single-site H_eff apply y=L.W.x.R, U(1), D=4096, charges -12..12"
                               if args.workload == "heff_d4096" else cfg["name"],
                   "precision": args.precision, "block_flops_per_step": flops,
                   "parallelism": "1 GPU"},
        "pct_fp64_mfma_peak": round(100.0 * value / PEAK["f64"], 2),
        "tiles": {f"step{i + 1}": list(plans[i][0].info()["tile"]) for i in mfma_steps},
        "tuning": tuning,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK[peak_key], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK[peak_key], 4), "traffic": None,
                     "kernel": "gemm grouped sector GEMM (steps 1 and 3)",
                     "avg_launch_us": round(gemm_avg_s * 1e6, 2)},
    }

    # parity spot check + CPU baseline: the oracle on the same inputs
    if not args.no_cpu_baseline:
        from oracle import blockwise
        from oracle.graded import Space, Structure
        osp = lambda s: Space(s.sectors, s.degs, s.dual)
        st = {k: Structure(cfg["tensors"][k]["sym"], [osp(s) for s in cfg["tensors"][k]["cod"]],
                           [osp(s) for s in cfg["tensors"][k]["dom"]]) for k in cfg["inputs"]}
        v0 = {k: synth.normal(st[k].size, cid, i) for i, k in enumerate(cfg["inputs"])}
        reps, spent, y_ref = 0, 0.0, None
        while spent < args.cpu_seconds and reps < 50:
            s2, v = dict(st), dict(v0)
            c0 = time.perf_counter()
            for out_, a, b, call in cfg["calls"]:
                s2[out_], v[out_] = blockwise.contract_storage(s2[a], v[a], call["pA"], call["qA"], s2[b], v[b],
                                                               call["pB"], call["qB"], call["pAB"], call["qAB"])
            spent += time.perf_counter() - c0
            reps += 1
            y_ref = v[cfg["output"]]
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
        except Exception:
            cores = os.cpu_count()
        out["cpu_baseline"] = {"value": round(flops * reps / spent / 1e12, 6), "unit": "TFLOP/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{reps} full H_eff applications of the same workload (numpy blockwise "
                                         f"fp64, OpenBLAS), {spent:.1f} s"}
        y = T[cfg["output"]].storage[: T[cfg["output"]].nelem].double().cpu().numpy()
        out["max_rel_err"] = float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))
        out["max_abs_rel_err_entry"] = float(np.max(np.abs(y - y_ref)) / np.max(np.abs(y_ref)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
