#!/usr/bin/env python
"""Benchmark of the Dense Inverse Search hot path on one MI355X.

Headline: one step = one whole pass of the method (pyramid, every scale's
inverse search, densification and refinement, upscaling) over one synthetic
1024x436 grayscale pair already resident in HBM, replayed from a HIP graph,
with the launch choices picked by the library's autotuner.  Also measured on
the same GPU: the second 1024x436 operating point, the batched form (64
pairs of uneven size per call) and the forward+backward form (8 pairs of
512x256, mean-EPE loss, gradients with respect to both frames).

Prints ONE JSON line: throughput in Mpix/s of dense output flow, a per-kernel
roofline entry for the kernel family that takes the most time (HIP events on
the library's stream), the parity of these very runs against the FP64
oracle, and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _layered(args):
    from paper_1603_03590_amd import synth
    w, h, disp, seed = args
    pr = synth.layered_pair(w, h, disp, seed)
    return pr.I0, pr.I1, pr.flow


def time_calls(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def roofline_of(stats):
    """Roofline entry of the kernel family with the largest summed event time:
    algorithmic bytes (flops for the search) per launch over its average
    launch duration, against the HBM (fp64 vector) peak."""
    top = sorted(stats, key=lambda k: -k["total_ms"])[0]
    avg_ms = top["total_ms"] / top["launches"]
    if top["name"] == "search":
        achieved = top["flops"] / top["launches"] / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP64_VECTOR_PEAK_TFLOPS)
    else:
        achieved = top["bytes"] / top["launches"] / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS)
    return roof, top, avg_ms


def kernel_table(stats, steps):
    out = {}
    for k in sorted(stats, key=lambda k: -k["total_ms"]):
        avg = k["total_ms"] / k["launches"]
        out[k["name"]] = dict(launches_per_step=k["launches"] / steps, us_per_step=k["total_ms"] * 1e3 / steps,
                              avg_launch_us=avg * 1e3,
                              GBps=(k["bytes"] / k["launches"]) / (avg * 1e-3) / 1e9,
                              GFLOPs=(k["flops"] / k["launches"]) / (avg * 1e-3) / 1e9)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the oracle CPU-baseline sample (0 disables it and the parity checks)")
    ap.add_argument("--op", default="c2a", choices=["c2a", "c2b"], help="operating point of the headline line")
    ap.add_argument("--batch", type=int, default=64, help="pairs in the batched measurement (0 skips it)")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline operating point (no launch-mode comparison, no second point); "
                         "for profiler runs")
    ap.add_argument("--tunables", default="",
                    help="skip the autotuner and fix the launch choices of the headline, e.g. 'tile=7,mode=1,lanes=16' "
                         "(for counter runs, where the profiler's serialisation would mislead the autotuner)")
    ap.add_argument("--only", default="all", choices=["all", "headline", "batched", "fwd_bwd", "hq"],
                    help="measure one part only (for profiler runs); 'headline' is --headline-only")
    ap.add_argument("--batch-tunables", default="",
                    help="skip the batch's autotuner and untuned timings and fix its launch choices, "
                         "e.g. 'tile=6,mode=1,lanes=0' (for counter runs)")
    ap.add_argument("--hq-tunables", default="",
                    help="skip the high-quality handles' autotuner and fix their launch choices (counter runs)")
    ap.add_argument("--hq-only", default="", help="run only this high-quality pair (c3a_1024x436 or c3b_2048x1024)")
    ap.add_argument("--fb-tunables", default="",
                    help="skip the forward+backward handles' autotuner and fix their launch choices (counter runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB five times (calibrates HBM counters)")
    ap.add_argument("--hq-steps", type=int, default=20,
                    help="timed steps of the high-quality configuration at 1024x436 and 2048x1024; 0 skips")
    ap.add_argument("--hq-parity", type=int, default=1,
                    help="check the high-quality flows against the oracle (1) or not (0)")
    ap.add_argument("--ext-steps", type=int, default=100,
                    help="timed steps of each extension (robust norms, stereo, forward-backward, colour); 0 skips")
    ap.add_argument("--fwd-bwd-pairs", type=int, default=8,
                    help="pairs of 512x256 in the forward+backward measurement (0 skips it)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues HIP may open for this process (GPU_MAX_HW_QUEUES, 1..32); the "
                         "forward+backward line runs its pairs on that many streams, and streams that share "
                         "a queue run one after the other")
    args = ap.parse_args()
    if args.only == "headline":
        args.headline_only = True
    part = lambda name: args.only in ("all", name)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU: the library has no multi-GPU path (pairs would shard across GPUs "
            "with no exchange); run it with --gpus 1")
        sys.exit(2)

    # read by the HIP runtime when the process first touches the GPU
    if not 1 <= args.hw_queues <= 32:
        log("--hw-queues takes 1..32")
        sys.exit(2)
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import numpy as np
    import torch
    from paper_1603_03590_amd import DIS, params, synth, _lib

    W, H = 1024, 436
    pr = synth.layered_pair(W, H, 100.0, 2)
    presets = {"c2a": 102, "c2b": 103}
    I0 = torch.from_numpy(pr.I0).cuda()
    I1 = torch.from_numpy(pr.I1).cuda()

    results = {}
    other = "c2b" if args.op == "c2a" else "c2a"
    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 5 copies of {args.copy_probe_mib} MiB")
        del src, dst
    for op in (() if not part("headline") else (args.op,) if args.headline_only else (args.op, other)):
        p = params(presets[op])
        d = DIS(p, W, H)
        out = torch.empty((2, H, W), device="cuda")
        flow = lambda: d.flow(I0, I1, out)
        modes = {}
        for name, mode in ((("phase", 1), ("persistent", 0)) if not args.headline_only else ()):
            d.set_tunables(None, 0, mode)
            modes[name] = time_calls(flow, args.steps, args.warmup) * 1e3
        if args.tunables:
            # fixed launch choices before the first flow, so that a profiled run
            # holds only launches of the measured configuration
            kv = dict(x.split("=") for x in args.tunables.split(","))
            lanes = int(kv.get("lanes", 0))
            d.set_tunables([lanes] * 16 if lanes else None, int(kv.get("tile", 7)), int(kv.get("mode", 1)))
        else:
            flow()
            d.autotune()
        tuned = d.tunables()
        dt = time_calls(flow, args.steps, args.warmup)
        f_tuned = out.cpu().numpy().astype(np.float64)
        # per-kernel event timing on the library's stream (tuned choices)
        _lib.dis_profile_enable(d.handle, True)
        for _ in range(3):
            flow()
        _lib.dis_profile_read(d.handle)
        for _ in range(args.profile_steps):
            flow()
        kstats = _lib.dis_profile_read(d.handle)
        _lib.dis_profile_enable(d.handle, False)
        d.close()
        results[op] = dict(ms=dt * 1e3, modes=modes, flow=f_tuned, kernels=kstats, tuned=tuned)
        log(f"[bench] {op}: tuned {dt * 1e3:.4f} ms/pair; untuned {modes}")

    if not part("headline"):
        head = None
    else:
        head = results[args.op]
        mpix = W * H / (head["ms"] * 1e-3) / 1e6
        # the paper's flow-only convention leaves out the pyramid (event-timed per step)
        pyr_ms = sum(k["total_ms"] for k in head["kernels"] if k["name"] == "pyramid") / args.profile_steps
        flow_only = dict(ms_per_step=head["ms"] - pyr_ms, value=W * H / ((head["ms"] - pyr_ms) * 1e-3) / 1e6,
                         unit="Mpix/s", excluded="pyramid (the Sobel gradients are computed inside the search)")
        roof, top, avg_ms = roofline_of(head["kernels"])
        # HBM traffic per launch of that kernel family, from the committed
        # counter summary when it was taken on these kernel sources with this
        # refinement tile (else null)
        traffic = None
        traffic_src = None
        from paper_1603_03590_amd import profsum
        is_ref = top["name"] == "refine"
        rec = profsum.read_traffic(os.path.join(ROOT, "profiles", f"{top['name']}_c2a_1024x436_hbm_traffic.md"),
                                   tile=head["tuned"]["refine_tile"] if is_ref else None,
                                   mode=head["tuned"]["launch_mode"] if is_ref else None)
        if rec and rec.get("source_sha") == profsum.source_hash():
            traffic = float(rec["bytes_per_launch"])
            traffic_src = f"profiles/{top['name']}_c2a_1024x436_hbm_traffic.md"
        roof.update(traffic=traffic, traffic_source=traffic_src, kernel=top["name"],
                    launches_per_step=top["launches"] / args.profile_steps,
                    avg_launch_us=avg_ms * 1e3, algorithmic_bytes_per_launch=top["bytes"] / top["launches"],
                    algorithmic_flops_per_launch=top["flops"] / top["launches"])

    # batched: 64 pairs of uneven sizes, one call per step
    batched = None
    bpairs = []
    if args.batch > 0 and part("batched"):
        sizes = synth.batch_sizes(args.batch, 4000)
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            bpairs = list(ex.map(_layered, [(w, h, 100.0, 1000 + k) for k, (w, h) in enumerate(sizes)]))
        log(f"[bench] generated {args.batch} pairs in {time.perf_counter() - t0:.1f} s")
        p = params(106)
        mw = max(w for w, _ in sizes)
        mh = max(h for _, h in sizes)
        d = DIS(p, mw, mh, max_batch=args.batch)
        bI0 = [torch.from_numpy(a).cuda() for a, _, _ in bpairs]
        bI1 = [torch.from_numpy(b).cuda() for _, b, _ in bpairs]
        bout = [torch.empty((2,) + a.shape, device="cuda") for a in bI0]
        call = lambda: d.flow_batched(bI0, bI1, bout)
        bmodes = {}
        if args.batch_tunables:
            kv = dict(x.split("=") for x in args.batch_tunables.split(","))
            lanes = int(kv.get("lanes", 0))
            d.set_tunables([lanes] * 16 if lanes else None, int(kv.get("tile", 7)), int(kv.get("mode", 1)))
        else:
            for name, mode in (("phase", 1), ("persistent", 0)):
                d.set_tunables(None, 0, mode)
                bmodes[name] = time_calls(call, max(5, args.steps // 20), 3) * 1e3
            call()
            d.autotune()
        bdt = time_calls(call, max(10, args.steps // 10), 3)
        torch.cuda.synchronize()
        # per-kernel event timing of the tuned batch (launches one by one)
        _lib.dis_profile_enable(d.handle, True)
        call()
        _lib.dis_profile_read(d.handle)
        for _ in range(3):
            call()
        bstats = _lib.dis_profile_read(d.handle)
        _lib.dis_profile_enable(d.handle, False)
        broof, btop, bavg = roofline_of(bstats)
        # counter bytes per launch of that kernel family in the committed
        # summary of this batch, while the sources and launch choices match
        from paper_1603_03590_amd import profsum
        btuned = d.tunables()
        b_is_ref = btop["name"] == "refine"
        bpath = f"profiles/{btop['name']}_c4_batch{args.batch}_hbm_traffic.md"
        brec = profsum.read_traffic(os.path.join(ROOT, bpath), tile=btuned["refine_tile"] if b_is_ref else None,
                                    mode=btuned["launch_mode"] if b_is_ref else None)
        btraffic = None
        if brec and brec.get("source_sha") == profsum.source_hash():
            btraffic = float(brec["bytes_per_launch"])
        broof.update(traffic=btraffic, traffic_source=bpath if btraffic is not None else None)
        broof.update(kernel=btop["name"], avg_launch_us=bavg * 1e3,
                     algorithmic_bytes_per_launch=btop["bytes"] / btop["launches"],
                     algorithmic_flops_per_launch=btop["flops"] / btop["launches"])
        pix = sum(w * h for w, h in sizes)
        # per-pair check on a sample: bitwise equal to the plain path
        sample = sorted(range(args.batch), key=lambda k: -sizes[k][0] * sizes[k][1])[:3]
        bit_equal = True
        for k in sample:
            h_, w_ = bpairs[k][0].shape
            dp = DIS(p, w_, h_)
            o = dp.flow(bI0[k], bI1[k])
            torch.cuda.synchronize()
            bit_equal &= bool(torch.equal(o, bout[k]))
            dp.close()
        btun = d.tunables()
        form = ("phase-major: one launch per phase of every level, all pairs in each" if btun["launch_mode"] & 1 else
                "persistent: one launch per level taking runs of tasks from a queue")
        batched = dict(value=pix / bdt / 1e6, unit="Mpix/s", ms_per_batch=bdt * 1e3, pairs=args.batch,
                       launch_form=form + " (the autotuner's pick; untuned_ms times both forms)",
                       output_mpix=pix / 1e6, untuned_ms={k: v for k, v in bmodes.items()},
                       plain_bitwise_equal_sample=bit_equal, tunables=d.tunables(),
                       kernels=kernel_table(bstats, 3), roofline=broof,
                       workload=f"{args.batch} layered pairs, sizes uniform over "
                                f"{{320x240, 640x480, 1024x436, 1280x720, 1920x1080}} (rng 4000), seeds 1000+k; "
                                f"patch 8, overlap 0.5, 16 GN iterations, scales auto..3, theta_vo = s+1")
        batched["_sample"] = sample
        batched["_out"] = {k: bout[k].cpu().numpy().astype(np.float64) for k in sample}
        d.close()
        log(f"[bench] batched: {bdt * 1e3:.3f} ms per {args.batch}-pair batch, {pix / bdt / 1e6:.0f} Mpix/s")

    # forward + loss + backward: 8 pairs of 512x256 (smooth bumps up to 16 px,
    # seeds 2000..2007), loss = mean end-point error against the ground truth,
    # dL/dI0 and dL/dI1 through the hand-written adjoint (autograd Function);
    # one handle per pair, so each pair's forward and backward replay their
    # own HIP graphs
    fwd_bwd = None
    fb_check = None
    if args.fwd_bwd_pairs > 0 and part("fwd_bwd"):
        from paper_1603_03590_amd import dis_flow
        nfb = args.fwd_bwd_pairs
        fbp = [synth.smooth_bump_pair(512, 256, 16.0, 2000 + k) for k in range(nfb)]
        pf = params(105, flags=_lib.DIS_FLAG_KEEP_FOR_BACKWARD)
        # one handle and one HIP stream per pair: the pairs' launch chains
        # are independent and run side by side on the GPU
        streams = [torch.cuda.Stream() for _ in range(nfb)]
        hs = [DIS(pf, 512, 256, stream=streams[k]) for k in range(nfb)]
        fI0 = [torch.from_numpy(q.I0).cuda().requires_grad_(True) for q in fbp]
        fI1 = [torch.from_numpy(q.I1).cuda().requires_grad_(True) for q in fbp]
        fgt = [torch.from_numpy(q.flow).cuda() for q in fbp]
        torch.cuda.synchronize()
        losses = [None] * nfb

        def fb_step():
            for k in range(nfb):
                with torch.cuda.stream(streams[k]):
                    fI0[k].grad = None
                    fI1[k].grad = None
                    f = dis_flow(fI0[k], fI1[k], hs[k])
                    L = torch.sqrt(((f - fgt[k]) ** 2).sum(0)).mean()
                    L.backward()
                    losses[k] = L

        def f_step():
            with torch.no_grad():
                for k in range(nfb):
                    with torch.cuda.stream(streams[k]):
                        f = hs[k].flow(fI0[k].detach(), fI1[k].detach())
                        losses[k] = torch.sqrt(((f - fgt[k]) ** 2).sum(0)).mean()

        f_step()
        for d_ in hs:
            if args.fb_tunables:
                kv = dict(x.split("=") for x in args.fb_tunables.split(","))
                lanes = int(kv.get("lanes", 0))
                d_.set_tunables([lanes] * 16 if lanes else None, int(kv.get("tile", 7)), int(kv.get("mode", 1)))
            else:
                d_.autotune()
        torch.cuda.synchronize()

        fsteps = max(10, args.steps // 5)
        t_fb = time_calls(fb_step, fsteps, max(3, args.warmup // 5))
        t_f = time_calls(f_step, fsteps, max(3, args.warmup // 5))
        # kernel time of the backward alone (events on the library's stream)
        for d_ in hs:
            _lib.dis_profile_enable(d_.handle, True)
        fb_step()
        for d_ in hs:
            _lib.dis_profile_read(d_.handle)
        for _ in range(3):
            fb_step()
        fb_k = {}
        for d_ in hs:
            for e in _lib.dis_profile_read(d_.handle):
                acc = fb_k.setdefault(e["name"], dict(name=e["name"], launches=0, total_ms=0.0, bytes=0.0, flops=0.0))
                for key in ("launches", "total_ms", "bytes", "flops"):
                    acc[key] += e[key]
            _lib.dis_profile_enable(d_.handle, False)
        torch.cuda.synchronize()
        fb_check = (fbp[0], fI0[0].grad.double().cpu().numpy(), fI1[0].grad.double().cpu().numpy(),
                    float(losses[0].detach()))
        mean_epe = float(torch.stack([l.detach() for l in losses]).mean())
        pix = nfb * 512 * 256
        fwd_bwd = dict(value=pix / t_fb / 1e6, unit="Mpix/s", ms_per_step=t_fb * 1e3, pairs=nfb,
                       forward_only=dict(value=pix / t_f / 1e6, ms_per_step=t_f * 1e3),
                       mean_epe_px=mean_epe, dtype_io="f32", streams=nfb, hw_queues=args.hw_queues,
                       tunables=hs[0].tunables(),
                       kernels=kernel_table(list(fb_k.values()), 3),
                       workload=f"{nfb} pairs 512x256 float32, smooth-bump generator (max 16 px, seeds "
                                f"2000..{2000 + nfb - 1}); patch 8, overlap 0.5, scales 3..0, "
                                f"16 GN iterations, theta_vo 3, theta_vi 5; loss = mean EPE vs ground truth; "
                                f"step = forward + loss + backward of every pair, one HIP stream per pair")
        for d_ in hs:
            d_.close()
        log(f"[bench] fwd+bwd: {t_fb * 1e3:.3f} ms per {nfb} pairs ({pix / t_fb / 1e6:.0f} Mpix/s); "
            f"forward only {t_f * 1e3:.3f} ms")

    # the high-quality configuration (patch 12, overlap 0.75, 128 GN iterations,
    # scales 4..0, theta_vo 5): the search's arithmetic dominates, so its
    # kernel's fp64 rate is the meaningful roofline there
    hq = {}
    if part("hq") and not args.headline_only and args.hq_steps > 0:
        for name, (w_, h_, seed) in (("c3a_1024x436", (1024, 436, 3)), ("c3b_2048x1024", (2048, 1024, 4))):
            if args.hq_only and name != args.hq_only:
                continue
            q = synth.layered_pair(w_, h_, 200.0, seed)
            d = DIS(params(104), w_, h_)
            a = torch.from_numpy(q.I0).cuda()
            b = torch.from_numpy(q.I1).cuda()
            o = torch.empty((2, h_, w_), device="cuda")
            call = lambda: d.flow(a, b, o)
            if args.hq_tunables:
                kv = dict(x.split("=") for x in args.hq_tunables.split(","))
                lanes = int(kv.get("lanes", 0))
                d.set_tunables([lanes] * 16 if lanes else None, int(kv.get("tile", 7)), int(kv.get("mode", 1)))
            else:
                call()
                d.autotune()
            t = time_calls(call, args.hq_steps, 3)
            _lib.dis_profile_enable(d.handle, True)
            call()
            _lib.dis_profile_read(d.handle)
            for _ in range(3):
                call()
            st = _lib.dis_profile_read(d.handle)
            _lib.dis_profile_enable(d.handle, False)
            r_, top_, avg_ = roofline_of(st)
            r_.update(kernel=top_["name"], avg_launch_us=avg_ * 1e3)
            hq[name] = dict(value=w_ * h_ / t / 1e6, unit="Mpix/s", ms_per_step=t * 1e3, tunables=d.tunables(),
                            kernels=kernel_table(st, 3), roofline=r_,
                            workload=f"layered pair {w_}x{h_}, rigid motion up to 200 px (seed {seed}); patch 12, "
                                     f"overlap 0.75, scales 4..0, 128 GN iterations, theta_vo 5, theta_vi 5",
                            _flow=o.cpu().numpy().astype(np.float64), _case=q)
            d.close()
            log(f"[bench] high quality {name}: {t * 1e3:.3f} ms/pair")

    # the paper's extensions (App. B, App. I) on the headline's frame size and
    # operating point: robust norms, stereo, forward-backward consistency,
    # colour frames; autotuned, graph replay, frames resident in HBM
    ext = {}
    if args.only == "all" and not args.headline_only and args.ext_steps > 0:
        hb = synth.smooth_bump_pair(W, H, 40.0, 2, horizontal=True)
        cb = synth.smooth_bump_pair(W, H, 40.0, 2, channels=3)
        cases = [
            ("l1", pr, dict(norm=_lib.DIS_NORM_L1), "layered pair of the headline, L1 search norm (App. B iii)"),
            ("huber", pr, dict(norm=_lib.DIS_NORM_HUBER),
             "layered pair of the headline, Huber search norm, b = 1 (App. B iii)"),
            ("stereo", hb, dict(flags=_lib.DIS_FLAG_STEREO),
             "smooth-bump pair 1024x436, horizontal motion up to 40 px (seed 2), 1-D search and refinement (App. I)"),
            ("fb_consistency", pr, dict(flags=_lib.DIS_FLAG_FB_CONSISTENCY),
             "layered pair of the headline, both directions with the merged densification (App. B ii)"),
            ("colour", cb, dict(flags=_lib.DIS_FLAG_COLOUR),
             "smooth-bump pair 1024x436, 3 correlated colour channels, motion up to 40 px (seed 2) (App. B i)"),
        ]
        for name, q, over, what in cases:
            pe = params(presets[args.op], **over)
            d = DIS(pe, W, H)
            a = torch.from_numpy(q.I0).cuda()
            b = torch.from_numpy(q.I1).cuda()
            o = torch.empty((2, H, W), device="cuda")
            call = lambda: d.flow(a, b, o)
            call()
            d.autotune()
            t = time_calls(call, args.ext_steps, max(3, args.warmup // 3))
            ext[name] = dict(value=W * H / t / 1e6, unit="Mpix/s", ms_per_step=t * 1e3,
                             workload=what + f"; operating point {args.op}", _flow=o.cpu().numpy().astype(np.float64),
                             _case=(q, pe))
            d.close()
            log(f"[bench] extension {name}: {t * 1e3:.4f} ms/pair")

    # parity of these runs and the CPU baseline (the FP64 oracle as it stands)
    parity = {}
    cpu = None
    if args.cpu_seconds > 0:
        from oracle import dis_oracle as O
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from dis_cases import oracle_params, parity as parity_stats

        def buckets(U, gt):
            # mean EPE over pixels whose true motion is under 10 px, 10-40 px, over 40 px
            e = np.sqrt(((U - gt) ** 2).sum(0))
            m = np.sqrt((gt ** 2).sum(0))
            out = {}
            for key, lo, hi in (("s0-10", 0.0, 10.0), ("s10-40", 10.0, 40.0), ("s40+", 40.0, np.inf)):
                sel = (m >= lo) & (m < hi)
                out[key] = float(e[sel].mean()) if sel.any() else None
            return out

        def check(name, U, I0n, I1n, gt, p):
            U_ref = O.dis_flow(torch.from_numpy(I0n), torch.from_numpy(I1n), oracle_params(p),
                               progress=lambda m: log(f"[bench] oracle for {name}: {m}")).numpy()
            frac, erel, dmax = parity_stats(U, U_ref, gt)
            epe = float(np.sqrt(((U - gt) ** 2).sum(0)).mean())
            parity[name] = {"frac_within_1e-2px": frac, "mean_epe_rel_diff": erel, "max_abs_diff_px": dmax,
                            "mean_epe_px": epe, "epe_buckets_gpu": buckets(U, gt),
                            "epe_buckets_oracle": buckets(U_ref, gt),
                            "passed": bool(frac >= 0.999 and erel <= 0.005)}

        for op, r in results.items():
            check(op, r["flow"], pr.I0, pr.I1, pr.flow, params(presets[op]))
        if batched:
            for k in batched["_sample"]:
                a, b, gt = bpairs[k]
                check(f"batched_pair{k}", batched["_out"][k], a, b, gt, params(106))
        if fb_check is not None:
            q, g0, g1, L = fb_check
            a = torch.from_numpy(q.I0).to(torch.float64).requires_grad_(True)
            b = torch.from_numpy(q.I1).to(torch.float64).requires_grad_(True)
            Lr = torch.sqrt(((O.dis_flow(a, b, oracle_params(params(105))) - torch.from_numpy(q.flow)) ** 2)
                            .sum(0)).mean()
            r0, r1 = torch.autograd.grad(Lr, (a, b))
            rel = lambda x, y: float(np.abs(x - y).max() / np.abs(y).max())
            parity["fwd_bwd_pair0"] = {"grad_I0_rel_max_err": rel(g0, r0.numpy()),
                                       "grad_I1_rel_max_err": rel(g1, r1.numpy()),
                                       "loss_rel_diff": abs(L / float(Lr) - 1.0),
                                       "passed": bool(rel(g0, r0.numpy()) <= 1e-4 and rel(g1, r1.numpy()) <= 1e-4)}
        for name, e in ext.items():
            q, pe = e["_case"]
            op_e = oracle_params(pe)
            if name == "colour":
                U_ref = O.dis_flow_colour(torch.from_numpy(q.I0), torch.from_numpy(q.I1), op_e).numpy()
            elif name == "fb_consistency":
                U_ref = O.dis_flow_fb(torch.from_numpy(q.I0), torch.from_numpy(q.I1), op_e)[0].numpy()
            else:
                U_ref = O.dis_flow(torch.from_numpy(q.I0), torch.from_numpy(q.I1), op_e).numpy()
            frac, erel, dmax = parity_stats(e["_flow"], U_ref, q.flow)
            parity[f"ext_{name}"] = {"frac_within_1e-2px": frac, "mean_epe_rel_diff": erel, "max_abs_diff_px": dmax,
                                     "passed": bool(frac >= 0.999 and erel <= 0.005)}
        # the high-quality runs against the oracle (the 2048x1024 pair takes
        # the oracle a few minutes: --hq-parity 0 leaves both out)
        if args.hq_parity:
            for name, e in hq.items():
                q = e["_case"]
                check(f"high_quality_{name}", e["_flow"], q.I0, q.I1, q.flow, params(104))
                log(f"[bench] parity high quality {name}: {parity[f'high_quality_{name}']['frac_within_1e-2px']:.6f}")
        op_p = oracle_params(params(presets[args.op]))
        t0 = time.perf_counter()
        runs = 0
        while True:
            O.dis_flow(torch.from_numpy(pr.I0), torch.from_numpy(pr.I1), op_p)
            runs += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        # the same on one thread (the paper's convention), for a bounded time
        nthr = torch.get_num_threads()
        torch.set_num_threads(1)
        t1 = time.perf_counter()
        runs1 = 0
        while True:
            O.dis_flow(torch.from_numpy(pr.I0), torch.from_numpy(pr.I1), op_p)
            runs1 += 1
            if time.perf_counter() - t1 >= max(2.0, args.cpu_seconds / 3):
                break
        el1 = time.perf_counter() - t1
        torch.set_num_threads(nthr)
        model = ""
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu = dict(value=runs * W * H / el / 1e6, unit="Mpix/s", cores=nthr, kind="oracle",
                   sample=f"{runs} full runs of the FP64 oracle on the same {W}x{H} pair ({el:.1f} s)",
                   single_thread=dict(value=runs1 * W * H / el1 / 1e6, runs=runs1, seconds=el1),
                   host=dict(cpu_model=model, nproc=os.cpu_count()))
    if batched:
        batched.pop("_sample")
        batched.pop("_out")
    for e in list(ext.values()) + list(hq.values()):
        e.pop("_flow")
        e.pop("_case")

    if head is None:
        # a part measured on its own (profiler runs): no headline line
        print(json.dumps({"only": args.only, "batched": batched, "fwd_bwd": fwd_bwd, "high_quality": hq or None}),
              flush=True)
        return

    cfg = dict(
        workload=f"plain DIS, one {W}x{H} grayscale float32 pair: layered scene (background + 6 textured "
                 f"rectangles, rigid motion up to 100 px, seed 2); "
                 + ("patch 8, overlap 0.3, 12 GN iterations" if args.op == "c2a" else
                    "patch 8, overlap 0.5, 16 GN iterations")
                 + "; scales 5..3, refinement theta_vo = s+1, theta_vi = 5; flow upscaled to full size",
        pairs_per_step=1, width=W, height=H, graph=True, autotuned=True,
    )
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
        "flow_only": flow_only,
        "cpu_baseline": cpu,
        "parity": parity,
        "kernels": kernel_table(head["kernels"], args.profile_steps),
        "untuned_ms_per_step": head["modes"],
        "tunables": head["tuned"],
        "other_operating_point": ({other: dict(ms_per_step=results[other]["ms"],
                                               value=W * H / (results[other]["ms"] * 1e-3) / 1e6,
                                               untuned_ms_per_step=results[other]["modes"])}
                                  if other in results else None),
        "batched": batched,
        "fwd_bwd": fwd_bwd,
        "extensions": ext or None,
        "high_quality": hq or None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
