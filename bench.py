#!/usr/bin/env python3
"""Throughput of the symmetric-contraction hot path on one MI355X.

Default workload (heff_d4096): one single-site effective-Hamiltonian
application y = L . W . x . R (three U(1) pairwise contractions, Alg.
"Single-site Benchmark") at virtual bond dimension D = 4096 over charges
-12..12, fp64.  A step is the whole application: for each contraction the
operand permutes, the grouped sector GEMM with its fused output scatter, the
small-K stream and the zero blocks.  Inputs are resident in HBM before the
timed region.  The same workload is then run with the fp32 and split-BF16x3
GEMM modes and their errors against the fp64 CPU oracle are reported.

Other workloads (--workload): heff_d1024; heff2_d1024 and heff2_d4096
(two-site effective Hamiltonian y = L . W . W . x2 . R, four contractions,
Alg. "Two-site Benchmark"); batch64 (64 independent
rank-3 x rank-4 contractions, one persistent grouped launch replayed from a
HIP graph, fp64 and fp32); peps (fermionic U(1) x fZ2 double layer
E = A^dagger o A interleaved to rank 8, D = 16); trace_d4096 (partial trace of
a U(1) tensor V (x) Wm <- V (x) Wm over the Wm pair, Alg. "Abelian Tensor
Trace", D = 4096); svd_d1024 (truncated SVD of the two-site tensor
x2 : V (x) P <- V (x) P* split between (a, p1) and (b, p2), D = 1024, 1024
values kept, Alg. "Abelian tensor decomposition").

Prints ONE JSON line.  value = useful block flops (sum over coupled charges
of 2 M N K) per second, whole job, with the whole application captured in
one HIP graph and replayed (the eager-launch time is reported beside it, and
the replayed result is checked equal to the eager one).  roofline = the
dominant kernel, timed with HIP events on its own stream inside an eager
timed region.  cpu_baseline =
the CPU oracle (numpy blockwise, fp64) timed on a bounded sample.
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
PEAK_KEY = {"native": "f64", "f32": "f32", "bf16x3": "bf16"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="heff_d4096", choices=["heff_d4096", "heff_d1024", "heff2_d1024", "heff2_d4096", "batch64", "peps",
                                                         "trace_d4096", "svd_d1024", "su2_d4096"])
    ap.add_argument("--precision", default="native", choices=["native", "f32", "bf16x3"])
    ap.add_argument("--no-variants", action="store_true", help="skip the fp32 / bf16x3 side runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile configuration")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned tile configurations (default: the one shipped with the package)")
    ap.add_argument("--retune", action="store_true",
                    help="time every tile configuration again and write the winners to the tune cache")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM byte counters)")
    return ap.parse_args()


PROFILE = os.path.join(ROOT, "profiles", "heff_d4096_all_kernels.md")
PROFILED_SOURCES = ["paper_2508_10076_amd/csrc/tk_kernels.hip", "paper_2508_10076_amd/csrc/tk_host.cpp",
                    "paper_2508_10076_amd/tuned_tiles.json"]


def profiled_traffic():
    """HBM bytes per GEMM-stage launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the plain-copy
    calibration), or None when the kernel sources, scheduler or tile table
    changed since the counters were taken."""
    import hashlib
    try:
        rec = None
        for line in open(PROFILE):
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
        h = hashlib.sha256()
        for src in PROFILED_SOURCES:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
    except (OSError, ValueError):
        return None
    if not rec or rec.get("sources_sha256") != h.hexdigest():
        return None
    return rec["traffic_bytes_per_launch"]


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:
        return os.cpu_count()


def np_abs(v):
    import numpy as np
    return np.abs(v)


def errors(np, got, ref, scale=None):
    """normwise |C - C*| / |C*|; entrywise max |C - C*|_ij / scale_ij (scale:
    the same computation on absolute values, |A||B|) and max |C - C*| / max |C*|."""
    d = np.abs(got - ref)
    out = {"normwise_rel_err": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
           "max_entry_err_rel_to_max": float(d.max() / np.abs(ref).max())}
    if scale is not None:
        nz = scale > 0
        out["max_rel_err"] = float(np.max(d[nz] / scale[nz])) if nz.any() else 0.0
    return out


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def one_thread():
    """Context limiting the BLAS pool to one thread (the paper's setting)."""
    from threadpoolctl import threadpool_limits
    return threadpool_limits(limits=1, user_api="blas")


def ostruct(t):
    from oracle.graded import Space, Structure
    osp = lambda s: Space(s.sectors, s.degs, s.dual)
    return Structure(t["sym"], [osp(s) for s in t["cod"]], [osp(s) for s in t["dom"]])


# ---------------------------------------------------------------------------
# H_eff application
# ---------------------------------------------------------------------------
class Heff:
    def __init__(self, tk, torch, cfg, cid, ctx, stream, precision, overlap=False):
        from paper_2508_10076_amd import synth
        self.tk, self.torch, self.cfg, self.stream = tk, torch, cfg, stream
        self.T = {}
        for i, k in enumerate(cfg["inputs"]):
            t = cfg["tensors"][k]
            self.T[k] = tk.tensor_create(ctx, t["sym"], t["cod"], t["dom"])
            self.T[k].storage[: self.T[k].nelem].copy_(torch.from_numpy(synth.normal(self.T[k].nelem, cid, i)))
        self.plans = []
        self.flops = 0.0
        for out, a, b, call in cfg["calls"]:
            T = self.T
            T[out] = tk.tensor_create_contracted(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"],
                                                 call["pAB"], call["qAB"])
            P = tk.Plan(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"], call["pAB"], call["qAB"],
                        T[out], precision=precision)
            info = P.info()
            self.flops += info["flops"]
            self.plans.append((P, T[a], T[b], T[out], info))
        # the MFMA-bound contractions: GEMMs with K well above the small-K limit
        self.mfma = [i for i, (P, *_r) in enumerate(self.plans) if P.gemms()[:, 2].max() > 64]
        # overlap=True: the operand permute of an input of the application
        # (here L, W, x, R) depends on nothing the step computes, so for every
        # contraction after the first it is enqueued on a second stream once
        # the first contraction's permutes are enqueued, and the main stream
        # waits for it just before that contraction's GEMM stage.  Measured on
        # the D = 4096 apply it does not pay (the persistent GEMM holds every
        # CU slot, so the side kernels mostly stretch it, and each cross-queue
        # dependency of the replayed graph costs ~5-10 us), so the timed step
        # runs on one stream; the test suite checks the overlapped schedule.
        inputs = set(cfg["inputs"]) if overlap else set()
        self.side = torch.cuda.Stream()
        self.side_stages, self.main_perm = {}, {}
        for i, (out, a, b, call) in enumerate(cfg["calls"]):
            ea, eb = i > 0 and a in inputs, i > 0 and b in inputs
            bits = (tk.STAGE_PERMUTE_A if ea else 0) | (tk.STAGE_PERMUTE_B if eb else 0)
            if bits:
                self.side_stages[i] = bits
            rest = (0 if ea else tk.STAGE_PERMUTE_A) | (0 if eb else tk.STAGE_PERMUTE_B)
            self.main_perm[i] = tk.STAGE_PERMUTE if rest == tk.STAGE_PERMUTE_A | tk.STAGE_PERMUTE_B else rest
        self.gemm_flops = sum(self.plans[i][4]["flops"] for i in self.mfma)
        torch.cuda.synchronize()

    def tune(self, precision, cache, force):
        from paper_2508_10076_amd import autotune
        tk, s = self.tk, self.stream
        out = {}
        for i in self.mfma:
            P, A, B, Cc, _ = self.plans[i]
            best, times = autotune.tune(P, lambda P=P, A=A, B=B, Cc=Cc: P.execute_stages(A, B, Cc, tk.STAGE_GEMM,
                                                                                           stream=s),
                                        P.gemms().tolist(), s, cache_path=cache, force=force,
                                        tag=("f64", precision))
            out[f"step{i + 1}"] = {"tile": list(best),
                                   "ms": {"x".join(map(str, c)): round(t, 4) for c, t in times.items()}}
        return out

    def step(self, ev=None):
        tk, torch, s, side = self.tk, self.torch, self.stream, self.side
        ready = {}
        for i, (P, A, B, Cc, _) in enumerate(self.plans):
            if self.main_perm[i]:
                P.execute_stages(A, B, Cc, self.main_perm[i], stream=s)
            if i == 0 and self.side_stages:
                # fork after the first contraction's permutes (which gate its
                # GEMM): the side work then fills the GEMM's tail instead of
                # competing with those permutes for bandwidth
                side.wait_stream(s)
                for j, bits in self.side_stages.items():
                    Pj, Aj, Bj, Cj, _ = self.plans[j]
                    Pj.execute_stages(Aj, Bj, Cj, bits, stream=side)
                    ready[j] = torch.cuda.Event()
                    ready[j].record(side)
            if i in ready:
                s.wait_event(ready[i])
            if ev is not None and i in self.mfma:
                ev.append(torch.cuda.Event(enable_timing=True))
                ev[-1].record(s)
                P.execute_stages(A, B, Cc, tk.STAGE_GEMM, stream=s)
                ev.append(torch.cuda.Event(enable_timing=True))
                ev[-1].record(s)
                P.execute_stages(A, B, Cc, tk.STAGE_ZERO, stream=s)
            else:
                P.execute_stages(A, B, Cc, tk.STAGE_GEMM | tk.STAGE_ZERO, stream=s)
        if self.side_stages:
            s.wait_stream(side)

    def run(self, steps, warmup):
        """Eager steps with HIP events around the GEMM stage of the MFMA-bound
        contractions (the roofline figure), then the same step captured in a
        HIP graph and replayed (the throughput figure: identical kernels,
        without host launch gaps)."""
        torch, s = self.torch, self.stream
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        evs = []
        t0.record(s)
        for _ in range(steps):
            self.step(evs)
        t1.record(s)
        torch.cuda.synchronize()
        eager_ms = t0.elapsed_time(t1)
        y_eager = self.output()
        gemm_ms = sum(evs[2 * j].elapsed_time(evs[2 * j + 1]) for j in range(len(evs) // 2))
        gemm_avg_s = gemm_ms / 1e3 / (len(evs) // 2)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.step()
        with torch.cuda.stream(s):
            for _ in range(warmup):
                g.replay()
        torch.cuda.synchronize()
        t0.record(s)
        with torch.cuda.stream(s):
            for _ in range(steps):
                g.replay()
        t1.record(s)
        torch.cuda.synchronize()
        total_ms = t0.elapsed_time(t1)
        same = bool((self.output() == y_eager).all())
        return dict(total_ms=total_ms, ms_per_step=total_ms / steps, eager_ms_per_step=eager_ms / steps,
                    graph_equals_eager=same, value=self.flops * steps / (total_ms / 1e3) / 1e12,
                    gemm_avg_us=gemm_avg_s * 1e6,
                    gemm_tflops=self.gemm_flops / len(self.mfma) / gemm_avg_s / 1e12)

    def output(self):
        y = self.T[self.cfg["output"]]
        return y.storage[: y.nelem].double().cpu().numpy()


def oracle_heff(cfg, cid, seconds, absolute=False):
    """The CPU oracle on the same inputs: (y, reps, seconds spent); with
    absolute=True on |inputs| (the entrywise error scale |L||W||x||R|)."""
    from oracle import blockwise
    from paper_2508_10076_amd import synth
    st = {k: ostruct(cfg["tensors"][k]) for k in cfg["inputs"]}
    v0 = {k: synth.normal(st[k].size, cid, i) for i, k in enumerate(cfg["inputs"])}
    if absolute:
        v0 = {k: np_abs(v) for k, v in v0.items()}
    reps, spent, y = 0, 0.0, None
    while (spent < seconds or reps == 0) and reps < 50:
        s2, v = dict(st), dict(v0)
        c0 = time.perf_counter()
        for out_, a, b, call in cfg["calls"]:
            s2[out_], v[out_] = blockwise.contract_storage(s2[a], v[a], call["pA"], call["qA"], s2[b], v[b],
                                                           call["pB"], call["qB"], call["pAB"], call["qAB"])
        spent += time.perf_counter() - c0
        reps += 1
        y = v[cfg["output"]]
    return y, reps, spent


def heff_workload(name):
    """(config, seed id, description, D, charge range) of an H_eff workload."""
    from paper_2508_10076_amd import synth
    return {
        "heff_d4096": (synth.config3, 3, "single-site H_eff apply y=L.W.x.R", 4096, 12),
        "heff_d1024": (synth.config2, 2, "single-site H_eff apply y=L.W.x.R", 1024, 8),
        "heff2_d1024": (lambda: synth.heff2_config(1024, 8, 3.0, 6), 6, "two-site H_eff apply y=L.W.W.x2.R", 1024, 8),
        "heff2_d4096": (lambda: synth.heff2_config(4096, 12, 4.5, 7), 7, "two-site H_eff apply y=L.W.W.x2.R",
                        4096, 12),
    }[name]


def bench_heff(args, tk, torch, np):
    make_cfg, cid, desc, D, qr = heff_workload(args.workload)
    cfg = make_cfg()
    ctx = tk.Context(0)
    stream = torch.cuda.Stream()
    H = Heff(tk, torch, cfg, cid, ctx, stream, args.precision)
    tuning = {} if args.no_tune else H.tune(args.precision, args.tune_cache, args.retune)
    torch.cuda.synchronize()
    r = H.run(args.steps, args.warmup)
    pk = PEAK_KEY[args.precision]
    out = {
        "metric": METRIC, "value": round(r["value"], 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "native" else args.precision,
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: {desc}, U(1), D={D}, charges -{qr}..{qr}",
                   "precision": args.precision, "block_flops_per_step": H.flops, "parallelism": "1 GPU"},
        "pct_fp64_mfma_peak": round(100.0 * r["value"] / PEAK["f64"], 2),
        "timing": {"mode": "HIP graph replay of the whole application (eager launches: see eager_ms_per_step)",
                   "eager_ms_per_step": round(r["eager_ms_per_step"], 5),
                   "graph_equals_eager": r["graph_equals_eager"]},
        "roofline": {"bound": "mfma", "achieved": round(r["gemm_tflops"], 4), "peak": PEAK[pk], "unit": "TFLOP/s",
                     "frac": round(r["gemm_tflops"] / PEAK[pk], 4),
                     "traffic": profiled_traffic() if (args.workload == "heff_d4096" and args.precision == "native")
                     else None,
                     "traffic_unit": "HBM bytes per launch",
                     "kernel": "grouped sector GEMM of the two MFMA-bound contractions (incl. split-K reduce)",
                     "avg_launch_us": round(r["gemm_avg_us"], 2)},
        "tiles": {f"step{i + 1}": list(H.plans[i][0].info()["tile"]) for i in H.mfma},
        "tuning": tuning,
    }
    y_gpu = H.output()
    variants = {}
    if not args.no_variants and args.precision == "native":
        for prec in ("f32", "bf16x3"):
            Hv = Heff(tk, torch, cfg, cid, ctx, stream, prec)
            if not args.no_tune:
                Hv.tune(prec, args.tune_cache, args.retune)
            rv = Hv.run(args.steps, args.warmup)
            variants[prec] = {"value": round(rv["value"], 4), "ms_per_step": round(rv["ms_per_step"], 5),
                              "gemm_tflops": round(rv["gemm_tflops"], 3),
                              "speedup_vs_fp64": round(r["ms_per_step"] / rv["ms_per_step"], 3),
                              "y": Hv.output()}
            del Hv
    if not args.no_cpu_baseline:
        y_ref, reps, spent = oracle_heff(cfg, cid, args.cpu_seconds)
        with one_thread():
            _, reps1, spent1 = oracle_heff(cfg, cid, args.cpu_seconds / 2)
        y_abs, _, _ = oracle_heff(cfg, cid, 0.0, absolute=True)
        out["cpu_baseline"] = {"value": round(H.flops * reps / spent / 1e12, 6), "unit": "TFLOP/s",
                               "cores": blas_threads(), "kind": "oracle",
                               "sample": f"{reps} full H_eff applications of the same workload (numpy blockwise "
                                         f"fp64, OpenBLAS), {spent:.1f} s",
                               "single_thread": {"value": round(H.flops * reps1 / spent1 / 1e12, 6),
                                                 "cores": 1, "sample": f"{reps1} applications, {spent1:.1f} s"},
                               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        out.update(errors(np, y_gpu, y_ref, y_abs))
        for prec, v in variants.items():
            v.update(errors(np, v.pop("y"), y_ref, y_abs))
    for v in variants.values():
        v.pop("y", None)
    if variants:
        out["precision_variants"] = variants
    return out


# ---------------------------------------------------------------------------
# batch of 64 contractions, one grouped launch replayed from a graph
# ---------------------------------------------------------------------------
def bench_batch(args, tk, torch, np):
    from paper_2508_10076_amd import autotune, synth
    cfg = synth.config4()
    call = cfg["call"]
    ctx = tk.Context(0)
    stream = torch.cuda.Stream()
    res, outs = {}, {}
    for dtype in ("f64", "f32"):
        plans, As, Bs, Cs, flops = [], [], [], [], 0.0
        for i, it in enumerate(cfg["items"]):
            A = tk.tensor_create(ctx, "U1", it["A"]["cod"], it["A"]["dom"], dtype=dtype)
            B = tk.tensor_create(ctx, "U1", it["B"]["cod"], it["B"]["dom"], dtype=dtype)
            A.storage[: A.nelem].copy_(torch.from_numpy(synth.normal(A.nelem, 4, 2 * i)))
            B.storage[: B.nelem].copy_(torch.from_numpy(synth.normal(B.nelem, 4, 2 * i + 1)))
            C = tk.tensor_create_contracted(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"],
                                            call["qAB"])
            P = tk.Plan(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"], call["qAB"], C)
            flops += P.info()["flops"]
            plans.append(P)
            As.append(A)
            Bs.append(B)
            Cs.append(C)
        batch = tk.Batch(ctx, plans, As, Bs, Cs)
        mnk = [g for P in plans for g in P.gemms().tolist()]
        best = None
        if not args.no_tune:
            best, _ = autotune.tune(batch, lambda: batch.launch(stream), mnk, stream, cache_path=args.tune_cache,
                                    force=args.retune, tag=(dtype, "native"))
        batch.capture(stream)

        def timed(fn, reps):
            with torch.cuda.stream(stream):
                for _ in range(args.warmup):
                    fn()
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_graph = timed(lambda: batch.replay(stream), args.steps)
        ms_seq = timed(lambda: [P.execute(A, B, C, stream=stream) for P, A, B, C in zip(plans, As, Bs, Cs)],
                       max(3, args.steps // 4))
        info = batch.info()
        res[dtype] = {"value": round(flops / ms_graph / 1e9, 4), "ms_per_step": round(ms_graph, 5),
                      "sequential_ms": round(ms_seq, 4), "speedup_vs_sequential": round(ms_seq / ms_graph, 3),
                      "ngemm": info["ngemm"], "ntiles": info["ntiles"], "tile": list(info["tile"]),
                      "block_flops": flops}
        batch.replay(stream)
        stream.synchronize()
        outs[dtype] = np.concatenate([C.storage[: C.nelem].double().cpu().numpy() for C in Cs])
        del batch, plans
    f64 = res["f64"]
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import blockwise

        def oracle_pass(absolute):
            ys = []
            for i, it in enumerate(cfg["items"]):
                stA, stB = ostruct(it["A"]), ostruct(it["B"])
                a, b = synth.normal(stA.size, 4, 2 * i), synth.normal(stB.size, 4, 2 * i + 1)
                if absolute:
                    a, b = np.abs(a), np.abs(b)
                ys.append(blockwise.contract_storage(stA, a, call["pA"], call["qA"], stB, b, call["pB"], call["qB"],
                                                     call["pAB"], call["qAB"])[1])
            return np.concatenate(ys)
        t0 = time.perf_counter()
        y_ref = oracle_pass(False)
        spent = time.perf_counter() - t0
        y_abs = oracle_pass(True)
        for dtype in res:
            res[dtype].update(errors(np, outs[dtype], y_ref, y_abs))
        cpu = {"value": round(f64["block_flops"] / spent / 1e12, 6), "unit": "TFLOP/s", "cores": blas_threads(),
               "kind": "oracle", "sample": f"one pass over the 64 contractions (numpy blockwise fp64, OpenBLAS), "
                                           f"{spent:.1f} s", "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    out = _batch_line(args, cfg, res, f64)
    if cpu:
        out["cpu_baseline"] = cpu
        out.update({k: f64[k] for k in ("normwise_rel_err", "max_rel_err", "max_entry_err_rel_to_max")})
    return out


def _batch_line(args, cfg, res, f64):
    return {"metric": METRIC, "value": f64["value"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": f64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{cfg['name']}: 64 U(1) contractions A[a;a',w] B[a',w,p;b], D~U{{256..2048}}, "
                                   f"one grouped launch in a HIP graph", "parallelism": "1 GPU"},
            "pct_fp64_mfma_peak": round(100 * f64["value"] / PEAK["f64"], 2),
            "roofline": {"bound": "mfma", "achieved": f64["value"], "peak": PEAK["f64"], "unit": "TFLOP/s",
                         "frac": round(f64["value"] / PEAK["f64"], 4), "traffic": None,
                         "kernel": "whole graph (permutes + grouped GEMM + reduce)"},
            "batch": res}


# ---------------------------------------------------------------------------
# fermionic PEPS double layer
# ---------------------------------------------------------------------------
def bench_peps(args, tk, torch, np):
    from paper_2508_10076_amd import synth
    cfg = synth.config5()
    call = cfg["call"]
    tA = cfg["tensors"]["A"]
    ctx = tk.Context(0)
    stream = torch.cuda.Stream()
    A = tk.tensor_create(ctx, tA["sym"], tA["cod"], tA["dom"])
    A.storage[: A.nelem].copy_(torch.from_numpy(synth.normal(A.nelem, 5, 0)))
    Ad = tk.tensor_adjoint(ctx, A)
    E = tk.tensor_create_contracted(ctx, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"],
                                    call["qAB"])
    res, samples = {}, {}
    pos = np.random.default_rng(51602).integers(0, E.nelem, size=200_000)
    pos_dev = torch.from_numpy(pos).cuda()
    for prec in ("native", "bf16x3"):
        P = tk.Plan(ctx, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"], call["qAB"], E,
                    precision=prec)
        flops = P.info()["flops"]

        def step():
            tk.tensor_adjoint(ctx, A, Ad, stream=stream)
            P.execute(Ad, A, E, stream=stream)
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                step()
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[prec] = {"ms_per_step": round(ms, 5), "value": round(flops / ms / 1e9, 5),
                     "gbps_output": round(8 * E.nelem / ms / 1e6, 1), "counts": P.counts()}
        samples[prec] = E.storage[pos_dev].double().cpu().numpy()
    nat = res["native"]
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle: the graph value of the network evaluated at the sampled
        # entries of E (pointwise definition, fp64), and the same sum of
        # |terms| as the entrywise error scale
        from oracle import blockwise, sampled
        stA = ostruct(tA)
        a = synth.normal(stA.size, 5, 0)
        t0 = time.perf_counter()
        sAd, bAd = blockwise.adjoint(stA, stA.to_blocks(a))
        Adn, Ax = sAd.to_dense(sAd.from_blocks(bAd)), stA.to_dense(a)
        free = [(0, i) for i in call["pA"]] + [(1, j) for j in call["qB"]]
        out_cod = [free[i] for i in call["pAB"]]
        pairs = [((0, x), (1, y)) for x, y in zip(call["qA"], call["pB"])]
        ocod, _ = sampled.graph_output_spaces([(sAd.cod, sAd.dom), (stA.cod, stA.dom)], out_cod, [])
        idx, size, off = sampled.codomain_channels("U1xFZ2", ocod)
        di = sampled.positions_to_dense(ocod, idx, size, off, pos)
        ref = sampled.graph_entries("U1xFZ2", [(Adn, sAd.cod, sAd.dom), (Ax, stA.cod, stA.dom)], pairs, out_cod,
                                    [], di)
        spent = time.perf_counter() - t0
        scale = np.zeros(pos.shape[0])
        for p in range(Ax.shape[0]):
            scale += np.abs(Adn[di[:, 0], di[:, 2], di[:, 4], di[:, 6], p]) * np.abs(Ax[p, di[:, 1], di[:, 3],
                                                                                      di[:, 5], di[:, 7]])
        for prec in res:
            res[prec].update(errors(np, samples[prec], ref, scale))
        cpu = {"value": round(pos.shape[0] / spent / 1e6, 4), "unit": "M entries/s", "cores": 1,
               "kind": "oracle", "sample": f"graph value of the double layer at {pos.shape[0]} uniformly drawn "
                                           f"entries of E (pointwise definition, numpy fp64), {spent:.1f} s; "
                                           f"errors are over the same entries",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    out = _peps_line(args, cfg, E, nat, res)
    if cpu:
        out["cpu_baseline"] = cpu
        out.update({k: nat[k] for k in ("normwise_rel_err", "max_rel_err", "max_entry_err_rel_to_max")})
    return out


def _peps_line(args, cfg, E, nat, res):
    return {"metric": METRIC, "value": nat["value"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": nat["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{cfg['name']}: E = A^dagger o A over P, interleaved rank 8, U(1)xfZ2, D=16",
                       "E_entries": E.nelem, "parallelism": "1 GPU"},
            "roofline": {"bound": "hbm", "achieved": nat["gbps_output"], "peak": HBM_PEAK, "unit": "GB/s",
                         "frac": round(nat["gbps_output"] / HBM_PEAK, 4), "traffic": None,
                         "kernel": "whole step (output write of E dominates)"},
            "peps": res}


def bench_trace(args, tk, torch, np):
    from paper_2508_10076_amd import synth
    q, d = synth.gaussian_degeneracies(4096, 12, 4.5)
    V = synth.u1_space(q, d)
    t = dict(sym="U1", cod=[V, synth.WM_U1], dom=[V, synth.WM_U1])
    ctx = tk.Context(0)
    stream = torch.cuda.Stream()
    A = tk.tensor_create(ctx, "U1", t["cod"], t["dom"])
    A.storage[: A.nelem].copy_(torch.from_numpy(synth.normal(A.nelem, 8, 0)))
    C = tk.tensor_create_traced(ctx, A, (0,), (2,), (1,), (3,))
    # algorithmic work: every diagonal element of A (traced indices equal) read once, C written once;
    # counted from the library's own channel table
    idx, _, _ = A.blocks()
    degs = [A.space(k)[1] for k in range(4)]
    diag = int(sum(degs[0][a] * degs[2][b] * degs[1][w] for a, w, b, w2 in idx if w == w2))
    nbytes = 8.0 * (diag + C.nelem)

    def step():
        tk.tensor_trace(ctx, A, (0,), (2,), (1,), (3,), C_=C, stream=stream)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"metric": METRIC, "value": round(diag / (ms * 1e-3) / 1e12, 5), "unit": "TFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "trace_u1_D4096: tr over Wm of A : V x Wm <- V x Wm, U(1), D=4096, "
                                   "charges -12..12", "A_entries": A.nelem, "C_entries": C.nelem,
                       "diagonal_entries": diag, "parallelism": "1 GPU"},
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK, "unit": "GB/s",
                         "frac": round(gbps / HBM_PEAK, 4), "traffic": None,
                         "kernel": "trace_kernel (diagonal of A read once, C written once)"}}


def bench_su2(args, tk, torch, np):
    from paper_2508_10076_amd import synth
    w = synth.su2_two_site(4096, 10, 4.0)
    plan = tk.SU2Plan(w["cod"], w["dom"], w["p"], w["q"])
    stream = torch.cuda.Stream()
    A = torch.from_numpy(synth.normal(plan.in_size, 9, 0)).cuda()
    C = torch.empty(plan.out_size, dtype=torch.float64, device="cuda")
    # algorithmic work: every input element read once, every output element written once
    nbytes = 8.0 * (plan.in_size + plan.out_size)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            plan.permute(A, C, stream=stream)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.permute(A, C, stream=stream)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gbps = nbytes / (ms * 1e-3) / 1e9
    dense = sum(d * (t + 1) for t, d in w["cod"][0])
    # the same tensor with its second physical leg bent to the domain
    # (V x P <- V x P*, the two-site matrix form): a transpose
    tp = tk.SU2Plan(w["cod"], w["dom"], [0, 1], [3, 2])
    Ct = torch.empty(tp.out_size, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            tp.permute(A, Ct, stream=stream)
    stream.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        tp.permute(A, Ct, stream=stream)
    e1.record(stream)
    e1.synchronize()
    ms_t = e0.elapsed_time(e1) / args.steps
    transpose = {"ms_per_step": round(ms_t, 5), "terms": tp.ncontrib,
                 "gbps": round(8.0 * (tp.in_size + tp.out_size) / (ms_t * 1e-3) / 1e9, 1),
                 "what": "x2 : V x P x P <- V bent to V x P <- V x P* (legs (0, 1 | 3, 2))"}
    return {"metric": "SU(2) leg permutation, algorithmic GB/s", "value": round(gbps, 2), "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "su2_two_site_D4096: swap of the two spin-1 legs of x2 : V x P x P <- V, "
                                   "SU(2), V = spins 0..10 with 4096 multiplets (dense dimension %d)" % dense,
                       "input_entries": plan.in_size, "output_entries": plan.out_size,
                       "recoupling_terms": plan.ncontrib, "parallelism": "1 GPU", "transpose": transpose,
                       "value_counts": "algorithmic bytes (input read once, output written once) per second"},
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK, "unit": "GB/s",
                         "frac": round(gbps / HBM_PEAK, 4), "traffic": None,
                         "kernel": "trace_kernel with no traced pairs (recoupling gather)"}}


def bench_svd(args, tk, torch, np):
    from paper_2508_10076_amd import synth
    cfg = synth.heff2_config(1024, 8, 3.0, 6)
    t = cfg["tensors"]["x"]
    ctx = tk.Context(0)
    stream = torch.cuda.Stream()
    A = tk.tensor_create(ctx, t["sym"], t["cod"], t["dom"])
    A.storage[: A.nelem].copy_(torch.from_numpy(synth.normal(A.nelem, 6, 0)))
    import time as _t
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup // 2)):
            U, S, Vh, err = tk.tensor_svd(ctx, A, (0, 1), (2, 3), max_dim=1024, stream=stream)
    steps = max(1, args.steps // 4)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            U, S, Vh, err = tk.tensor_svd(ctx, A, (0, 1), (2, 3), max_dim=1024, stream=stream)
    torch.cuda.synchronize()
    ms = (_t.perf_counter() - t0) * 1e3 / steps
    with torch.cuda.stream(stream):
        sweeps = tk.tensor_svd(ctx, A, (0, 1), (2, 3), max_dim=1024, stream=stream, info=True)[4]["max_sweeps"]
    nbytes = 8.0 * (A.nelem + U.nelem + S.nelem + Vh.nelem)
    _, rows, cols, _ = A.sectors()  # the split (a, p1) | (b, p2) is the stored matrix form
    mn = [(int(max(r, c)), int(min(r, c))) for r, c in zip(rows, cols)]
    gbps = nbytes / (ms * 1e-3) / 1e9
    flops = sum(4.0 * m * n * n for m, n in mn)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's truncated SVD of the same tensor (permute, per-sector
        # LAPACK SVD, truncation, factor assembly), as many runs as fit the
        # CPU budget
        from oracle import decomp
        st, x = ostruct(t), synth.normal(A.nelem, 6, 0)
        reps, t1 = 0, _t.perf_counter()
        while True:
            decomp.svd_trunc(st, x, (0, 1), (2, 3), 1024)
            reps += 1
            if _t.perf_counter() - t1 > args.cpu_seconds / 4 or reps >= 50:
                break
        spent = _t.perf_counter() - t1
        cpu = {"value": round(flops / (spent / reps) / 1e12, 6), "unit": "TFLOP/s", "cores": blas_threads(),
               "kind": "oracle", "ms_per_decomposition": round(spent / reps * 1e3, 2),
               "sample": f"{reps} full truncated SVDs of the same tensor (numpy, LAPACK per sector), {spent:.1f} s",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    return {"metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e12, 6),
            "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": max(1, args.warmup // 2),
            "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "svd_u1_D1024: truncated SVD of x2 : V x P <- V x P*, (a, p1) | (b, p2), "
                                   "D=1024, 1024 kept", "sectors": len(mn), "largest_block": max(mn),
                       "truncation_error": err, "jacobi_sweeps": sweeps, "parallelism": "1 GPU",
                       "value_counts": "4 m n^2 per sector matrix (the singular values of an m x n block)"},
            "roofline": {"bound": "hbm", "achieved": round(gbps, 2), "peak": HBM_PEAK, "unit": "GB/s",
                         "frac": round(gbps / HBM_PEAK, 5), "traffic": None,
                         "kernel": "whole decomposition (block-Jacobi rounds, one launch per round; host sync "
                                   "after every sweep)"},
            "cpu_baseline": cpu}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2508_10076_amd import autotune, tk
    if args.tune_cache is None:
        args.tune_cache = autotune.DEFAULT_CACHE
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.randn(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload.startswith("heff"):
        out = bench_heff(args, tk, torch, np)
    elif args.workload == "batch64":
        out = bench_batch(args, tk, torch, np)
    elif args.workload == "trace_d4096":
        out = bench_trace(args, tk, torch, np)
    elif args.workload == "svd_d1024":
        out = bench_svd(args, tk, torch, np)
    elif args.workload == "su2_d4096":
        out = bench_su2(args, tk, torch, np)
    else:
        out = bench_peps(args, tk, torch, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
