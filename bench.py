#!/usr/bin/env python
"""Benchmark of the Dense Inverse Search hot path on one MI355X.

One step = one whole pass of the method (pyramid, every scale's inverse
search, densification and refinement, upscaling) over one synthetic
1024x436 grayscale pair already resident in HBM, replayed from a HIP graph.
Prints ONE JSON line with the throughput in Mpix/s of dense output flow,
a per-kernel roofline entry for the kernel that takes the most time
(measured with HIP events on the library's stream), the parity of this very
run against the FP64 oracle, and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the oracle CPU-baseline sample (0 disables it)")
    ap.add_argument("--op", default="c2a", choices=["c2a", "c2b"], help="operating point of the headline line")
    ap.add_argument("--profile-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU: this build has no multi-GPU path (pairs would shard across GPUs "
            "with no exchange); run it with --gpus 1")
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1603_03590_amd import DIS, params, synth, _lib

    W, H = 1024, 436
    pr = synth.layered_pair(W, H, 100.0, 2)
    presets = {"c2a": 102, "c2b": 103}
    I0 = torch.from_numpy(pr.I0).cuda()
    I1 = torch.from_numpy(pr.I1).cuda()

    results = {}
    for op in (args.op, "c2b" if args.op == "c2a" else "c2a"):
        p = params(presets[op])
        d = DIS(p, W, H)
        out = torch.empty((2, H, W), device="cuda")
        for _ in range(args.warmup):
            d.flow(I0, I1, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            d.flow(I0, I1, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        flow = out.cpu().numpy().astype(np.float64)
        # per-kernel event timing on the library's stream
        _lib.dis_profile_enable(d.handle, True)
        for _ in range(3):
            d.flow(I0, I1, out)
        _lib.dis_profile_read(d.handle)          # discard the first eager passes
        for _ in range(args.profile_steps):
            d.flow(I0, I1, out)
        kstats = _lib.dis_profile_read(d.handle)
        _lib.dis_profile_enable(d.handle, False)
        eager_t0 = time.perf_counter()
        p_e = params(presets[op], flags=_lib.DIS_FLAG_NO_GRAPH)
        de = DIS(p_e, W, H)
        for _ in range(args.warmup):
            de.flow(I0, I1, out)
        torch.cuda.synchronize()
        eager_t0 = time.perf_counter()
        for _ in range(args.steps):
            de.flow(I0, I1, out)
        torch.cuda.synchronize()
        dt_eager = (time.perf_counter() - eager_t0) / args.steps
        de.close()
        d.close()
        results[op] = dict(ms=dt * 1e3, ms_eager=dt_eager * 1e3, flow=flow, kernels=kstats, params=p.as_dict())
        log(f"[bench] {op}: {dt * 1e3:.4f} ms/pair (graph), {dt_eager * 1e3:.4f} ms/pair (eager)")

    head = results[args.op]
    mpix = W * H / (head["ms"] * 1e-3) / 1e6

    # roofline of the kernel family with the largest total time
    ks = sorted(head["kernels"], key=lambda k: -k["total_ms"])
    top = ks[0]
    avg_ms = top["total_ms"] / top["launches"]
    per_launch_bytes = top["bytes"] / top["launches"]
    per_launch_flops = top["flops"] / top["launches"]
    if top["name"] == "search":
        achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP64_VECTOR_PEAK_TFLOPS)
    else:
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS)
    roof.update(kernel=top["name"], launches_per_step=top["launches"] // args.profile_steps,
                avg_launch_us=avg_ms * 1e3, traffic=None)
    kernel_table = {k["name"]: dict(launches_per_step=k["launches"] / args.profile_steps,
                                    us_per_step=k["total_ms"] * 1e3 / args.profile_steps,
                                    avg_launch_us=k["total_ms"] * 1e3 / k["launches"],
                                    GBps=(k["bytes"] / k["launches"]) / (k["total_ms"] / k["launches"] * 1e-3) / 1e9,
                                    GFLOPs=(k["flops"] / k["launches"]) / (k["total_ms"] / k["launches"] * 1e-3) / 1e9)
                    for k in ks}

    # parity of this run and the CPU baseline (the FP64 oracle as it stands)
    parity = {}
    cpu = None
    if args.cpu_seconds > 0:
        from oracle import dis_oracle as O
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from dis_cases import oracle_params, parity as parity_stats
        for op, r in results.items():
            U_ref = O.dis_flow(torch.from_numpy(pr.I0), torch.from_numpy(pr.I1),
                               oracle_params(params(presets[op]))).numpy()
            frac, erel, dmax = parity_stats(r["flow"], U_ref, pr.flow)
            epe = float(np.sqrt(((r["flow"] - pr.flow) ** 2).sum(0)).mean())
            parity[op] = {"frac_within_1e-2px": frac, "mean_epe_rel_diff": erel, "max_abs_diff_px": dmax,
                          "mean_epe_px": epe, "passed": bool(frac >= 0.999 and erel <= 0.005)}
        op_p = oracle_params(params(presets[args.op]))
        t0 = time.perf_counter()
        runs = 0
        while True:
            O.dis_flow(torch.from_numpy(pr.I0), torch.from_numpy(pr.I1), op_p)
            runs += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        cpu = dict(value=runs * W * H / el / 1e6, unit="Mpix/s", cores=torch.get_num_threads(), kind="oracle",
                   sample=f"{runs} full runs of the FP64 oracle on the same {W}x{H} pair ({el:.1f} s)")

    cfg = dict(
        workload=f"plain DIS, one {W}x{H} grayscale float32 pair: layered scene (background + 6 textured "
                 f"rectangles, rigid motion up to 100 px, seed 2); "
                 + ("patch 8, overlap 0.3, 12 GN iterations" if args.op == "c2a" else
                    "patch 8, overlap 0.5, 16 GN iterations")
                 + "; scales 5..3, refinement theta_vo = s+1, theta_vi = 5; flow upscaled to full size",
        pairs_per_step=1, width=W, height=H, graph=True,
    )
    other = "c2b" if args.op == "c2a" else "c2a"
    line = {
        "metric": "flow Mpix/s @1024x436 (EPE-matched to oracle)",
        "value": mpix,
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "kernels": kernel_table,
        "eager_ms_per_step": head["ms_eager"],
        "other_operating_point": {other: dict(ms_per_step=results[other]["ms"],
                                              value=W * H / (results[other]["ms"] * 1e-3) / 1e6,
                                              eager_ms_per_step=results[other]["ms_eager"])},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
