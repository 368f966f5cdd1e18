"""Benchmark of the two-table Figaro hot path on one MI355X.

One step = the whole path on one batch of synthetic input already resident in
HBM: key grouping, head/tail scans, compact-matrix assembly, Householder TSQR
(leaves, tree, merge, sign) -> R, then one-sided Jacobi -> sigma.

Workload: Cartesian product of two 1e5 x 32 FP64 N(0,1) tables (a 1e10 x 64
join that is never materialised).  Six forms are timed: the Claim 1 compact
matrix and the two-sided form, each with an FP64 reduction, an FP32 one, and
an FP32 one followed by the FP64 refinement sweep.  `value`
is the fastest form whose R and sigma are within 1e-5 of the oracle; every
form is listed under "forms".  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "R+σ latency & effective join rows/s: FP32-MFMA batched vs FP64, rel err ≤1e-5"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
TOL = 1e-5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="claim1:fp64,two_sided:fp64,claim1:fp32,two_sided:fp32,"
                                       "claim1:fp32_refine,two_sided:fp32_refine")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch

    import paper_2503_23385_amd as fg
    from paper_2503_23385_amd import workloads as W

    if not os.path.exists(fg.LIB_PATH):
        from paper_2503_23385_amd import build as hb
        hb.build()
    dev = torch.device("cuda:0")
    inst = W.config2()
    m1, n1 = inst.A.shape
    m2, n2 = inst.B.shape
    N = n1 + n2
    join_rows = m1 * m2
    A = torch.from_numpy(inst.A).to(dev)
    B = torch.from_numpy(inst.B).to(dev)
    stream = torch.cuda.current_stream()

    # Oracle: reference result for the error columns, and the CPU baseline timing.
    Ro = So = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
            oracle.build()
        t0 = time.perf_counter()
        reps = 0
        while True:
            Ro = oracle.r(inst)
            So = oracle.sigma(Ro)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or reps >= 20:
                break
        cpu = {"value": join_rows * reps / el, "unit": "join rows/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{reps} full run(s) of the FP64 CPU oracle (groups, compact matrix, Householder QR, "
                         f"Jacobi) on the same 1e5x32 + 1e5x32 workload, {el:.1f} s"}

    forms = {}
    for spec in args.forms.split(","):
        layout, prec = spec.split(":")
        two = layout == "two_sided"
        ws = fg.alloc_workspace(fg.r_workspace_size(A, B, None, None, prec, two), dev)
        R = torch.empty((N, N), dtype=torch.float64, device=dev)
        S = torch.empty(N, dtype=torch.float64, device=dev)
        sws = fg.alloc_workspace(256, dev)

        def step():
            fg.r(A, B, None, None, prec, ws=ws, out=R, two_sided=two)
            fg.sigma(R, out=S, ws=sws)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        assert fg.status(ws) == 0
        # Timed region: K steps bracketed by synchronisation, HIP events on the launch stream.
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        # The same K steps again with per-stage events (library stage timing).
        fg.timing_enable(True)
        fg.timing_read()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        stages = fg.timing_read()
        fg.timing_enable(False)
        stage_ms = {k: v[0] / args.steps for k, v in stages.items()}
        launches = {k: v[1] / args.steps for k, v in stages.items()}
        sweeps = int(sws[:4].view(torch.int32)[0].item())
        errs = None
        if Ro is not None:
            Rg, Sg = R.cpu().numpy(), S.cpu().numpy()
            errs = {"R_relF": float(np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)),
                    "sigma_rel2": float(np.linalg.norm(Sg - So) / np.linalg.norm(So))}
        forms[spec] = {"ms_per_step": ms, "value": join_rows / (ms / 1e3), "stage_ms": stage_ms,
                       "launches_per_step": launches, "errors_vs_oracle": errs, "jacobi_sweeps": sweeps,
                       "layout": layout, "precision": prec}
        del ws, R, S

    ok = [k for k, f in forms.items()
          if f["errors_vs_oracle"] is None
          or (f["errors_vs_oracle"]["R_relF"] <= TOL and f["errors_vs_oracle"]["sigma_rel2"] <= TOL)]
    chosen = min(ok, key=lambda k: forms[k]["ms_per_step"])
    f = forms[chosen]

    # Dominant kernel of the chosen form and its algorithmic work per launch.
    esz = 8 if f["precision"] == "fp64" else 4
    peak_tsqr = PEAK_FP64_TFLOPS if f["precision"] == "fp64" else PEAK_FP32_TFLOPS
    two = f["layout"] == "two_sided"
    work = {
        # B read once per pass of the scan (FP64) + region 2 written once
        "scan": ("hbm", (m2 * n2 * 8 + (m2 - 1) * n2 * esz + (m1 * n1 * 8 + (m1 - 1) * n1 * esz if two else 0)) / 1e9),
        "assemble": ("hbm", (m1 * n1 * 8 + m1 * N * esz) / 1e9 if not two else (N * esz) / 1e9),
        # streaming `rows` rows of width w into a w x w triangle costs 2 w^2 flops per row
        "tsqr_m1": ("alu", 2.0 * m1 * N * N / 1e12),
        "tsqr_m2": ("alu", 2.0 * (m2 - 1) * n2 * n2 / 1e12),
        "tsqr_ta": ("alu", 2.0 * (m1 - 1) * n1 * n1 / 1e12),
        "tsqr_tb": ("alu", 2.0 * (m2 - 1) * n2 * n2 / 1e12),
        # both tail regions of the two-sided form in one launch
        "tsqr_tails": ("alu", 2.0 * ((m1 - 1) * n1 * n1 + (m2 - 1) * n2 * n2) / 1e12),
        # one sweep: n(n-1)/2 pairs, 3 dot products and a rotation of two n-vectors (12 n flops)
        "jacobi": ("alu", 6.0 * N * N * (N - 1) * f["jacobi_sweeps"] / 1e12),
    }
    stage_ms = f["stage_ms"]
    dom = max((k for k in stage_ms if k in work), key=lambda k: stage_ms[k])
    per_launch_ms = stage_ms[dom] / max(1.0, f["launches_per_step"][dom])
    bound, amount = work[dom]
    t = per_launch_ms / 1e3
    if bound == "hbm":
        roof = {"kernel": dom, "bound": "hbm", "achieved": amount / t, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": amount / t / PEAK_HBM_GBS, "traffic": None}
    else:
        # the FP32 forms' TSQR updates run in FP32; Jacobi always runs in FP64
        peak_alu = PEAK_FP64_TFLOPS if dom == "jacobi" else peak_tsqr
        roof = {"kernel": dom, "bound": "alu", "achieved": amount / t, "peak": peak_alu,
                "unit": "TFLOP/s", "frac": amount / t / peak_alu, "traffic": None}

    line = {
        "metric": METRIC,
        "value": f["value"],
        "unit": "join rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_refine": "f32+f64"}[f["precision"]],
        "data": "synthetic",
        "config": {"workload": "cartesian product, A and B 1e5 x 32 FP64 N(0,1), join 1e10 x 64 "
                               "(never materialised), R 64x64 + sigma",
                   "join_rows": join_rows, "form": chosen},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
