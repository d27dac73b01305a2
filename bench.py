"""Batched partial-delivery render benchmark (one MI355X).

Step = one pass of the whole hot path over one batch of synthetic input:
deformation + projection of every Gaussian, depth sort, tile binning and
per-tile lists (dgs_bin), then masked compositing of every delivery state
(dgs_composite).  Inputs are resident in HBM before timing starts.  The
headline's K steps rotate over three streams, each step on a workspace of its
own, so one step's binning overlaps the compositing of the steps before it;
the same K steps on one stream are reported beside it.

Prints ONE JSON line: batched delivery-states/s (value), the plain per-state
render timed one state at a time with a synchronisation after each, fwd+bwd ms/iter on the
250k-Gaussian 720p 8-state training workload, the compositing kernel's
roofline, and the oracle's CPU rate on a bounded sample.
"""

from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "delivery-states rendered/s batched vs per-state; fwd+bwd ms/iter @250k G"
PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak (counts packed FP32 FMA)
# Without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic FLOPs (an FMA counts 2) per unit of compositing work:
FLOPS_PER_ALPHA = 14       # dx, dy, quadratic form (8), scale, exp, x opacity, cap
FLOPS_PER_BLEND = 8        # T*alpha, 3 FMA colour, T - T*alpha
# Backward compositing, per alpha evaluation: the forward's 14 + dq = dL/dalpha alpha ln2 (2) + the
# six per-pixel terms of (u, v, A', B', C', log2 o) (16) + the pixel sums of the nine 2D gradients (9)
FLOPS_BWD_PER_ALPHA = 41
# per blend: the forward's 8 + g . c (5) + colour-behind update (2) + dL/dalpha (4) + dL/dc (6)
FLOPS_BWD_PER_BLEND = 25
LAUNCH = {"auto": None, "grid": False, "persistent": True}
PIPELINE_DEPTH = 3  # streams (each with its own workspace) the headline's steps rotate over
# the kernels one dgs_backward call launches on the training workload (their traffic record)
BWD_KERNELS = "k_composite_bwd<8,16,16>+k_geometry_bwd<false>"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="g250k_800px_64states")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--states-per-group", type=int, default=8)
    ap.add_argument("--launch", choices=("auto", "grid", "persistent"), default="auto",
                    help="compositing launch: one workgroup per work item, or resident workgroups "
                         "draining per-XCD work queues (auto: the library decides)")
    ap.add_argument("--no-per-state", action="store_true")
    ap.add_argument("--no-fwdbwd", action="store_true")
    ap.add_argument("--no-train-step", action="store_true", help="skip the Eq. (2) training-step leg")
    ap.add_argument("--no-serial-fwdbwd", action="store_true",
                    help="skip the 2.7M-Gaussian fwd+bwd leg: 32 states batched vs one state per call")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2.7M-Gaussian 256-state leg and the 32,768-state PSNR sweep")
    ap.add_argument("--no-utility", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batch-size sweep of the headline scene")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the leg with attribute refinement levels on the same workload")
    ap.add_argument("--utility", default="g1m_540p_utility_64groups_16contexts",
                    help="counterfactual-utility workload timed beside the main metric")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graph", action="store_true", help="time replays of one captured HIP graph")
    ap.add_argument("--tune", action="store_true",
                    help="pick tile shape, states per group, launch and LDS batch by timing")
    ap.add_argument("--lds-batch", type=int, default=256, choices=(128, 256, 512),
                    help="list entries staged in LDS per compositing batch")
    ap.add_argument("--streams", type=int, default=PIPELINE_DEPTH,
                    help="streams (each with its own workspace) the timed steps rotate over; 1 times the "
                         "steps on one stream only")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (delivery states would "
              "shard across GPUs, each rendering its share with no exchange in the forward)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_2606_17212_amd as dgs
    from paper_2606_17212_amd import profile_summary

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    tw, th = (int(x) for x in args.tile.split("x"))
    w = synth.make_workload(args.workload)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(w.codes).to(dev)
    W = int(codes.shape[0])
    bg = tuple(float(x) for x in w.background)
    if w.total_states:
        return psnr_sweep(args, w, scene, cam, dgs, torch, np, dev, tw, th)
    if args.tune:
        res = dgs.Autotuner().tune(scene, cam, codes, w.basis, bg, reps=3)
        (tw, th), args.states_per_group = res.tile, res.states_per_group
        args.launch = "persistent" if res.persistent else "grid"
        args.lds_batch = res.lds_batch
        log(f"[bench] autotuner: {tw}x{th}, S={args.states_per_group}, {args.launch}, LDS batch {args.lds_batch} "
            f"({res.ms:.3f} ms); "
            f"table {res.table}")
    r = dgs.Renderer(dev, tile=(tw, th), states_per_group=args.states_per_group, persistent=LAUNCH[args.launch],
                     lds_batch=args.lds_batch)
    M = r.plan(scene, cam, w.basis, W)
    log(f"[bench] {args.workload}: N={scene.n} {cam.width}x{cam.height} W={W} instances={M}")
    img = torch.empty((W, cam.height, cam.width, 3), dtype=torch.float32, device=dev)

    graph = dgs.CapturedRender(r, scene, cam, codes, w.basis, bg) if args.graph else None
    if graph is not None:
        img = graph.out

    def step():
        if graph is not None:
            graph.replay()
            return
        r.bin(scene, cam, w.basis)
        r.composite(scene, cam, codes, w.basis, bg, out=img)

    for _ in range(args.warmup):
        step()
    r.check()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    # every event recorded once before the timed region (the runtime creates an event on its first record)
    for e in [x for row in ev for x in row] + [t_start, t_end]:
        e.record(st)
    torch.cuda.synchronize()
    # no Python garbage collection inside the timed loops: a full collection can stall the host for
    # tens of milliseconds, leaving the device idle between launches
    gc.collect()
    gc.disable()
    if graph is not None:
        t_start.record(st)
        for k in range(args.steps):
            graph.replay()
        t_end.record(st)
        torch.cuda.synchronize()
    # eager pass with events around each half (also the timed region without a graph)
    t0, t1 = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    t0.record(st)
    t1.record(st)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    t0.record(st)
    for k in range(args.steps):
        ev[k][0].record(st)
        r.bin(scene, cam, w.basis)
        ev[k][1].record(st)
        r.composite(scene, cam, codes, w.basis, bg, out=img)
        ev[k][2].record(st)
    t1.record(st)
    host_ms = (time.perf_counter() - h0) * 1e3  # time the host took to enqueue the timed steps
    torch.cuda.synchronize()
    if graph is None:
        t_start, t_end = t0, t1
    total_ms = t_start.elapsed_time(t_end)
    bin_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    comp_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    ms_step = total_ms / args.steps
    value = W * args.steps / (total_ms / 1e3)
    r.check()
    log(f"[bench] batched: {ms_step:.3f} ms/step (bin {bin_ms:.3f}, composite {comp_ms:.3f}) -> {value:.1f} states/s")
    # two more independent timed repetitions of the same K steps (the paper's
    # protocol: three repetitions, Student-t interval over them)
    reps = [value]
    for _ in range(2):
        step()  # one untimed step before each repetition
        torch.cuda.synchronize()
        t0.record(st)
        for k in range(args.steps):
            step()
        t1.record(st)
        torch.cuda.synchronize()
        reps.append(W * args.steps / (t0.elapsed_time(t1) / 1e3))
    r.check()
    # median of the three repetitions (the paper's protocol), robust to a host hiccup in one of them;
    # the first repetition's per-step split is kept beside it
    first_value = value
    serial_value = float(np.median(reps))
    log(f"[bench] batched, one stream, median of {len(reps)} repetitions: {W / serial_value * 1e3:.3f} ms/step "
        f"-> {serial_value:.1f} states/s")
    # The headline: the same K steps, each the whole path (binning, then compositing), issued round
    # robin on --streams streams with a renderer (workspace) per stream.  A step's binning, a
    # chain of short launches that leave most of the chip idle, and the last workgroups of its
    # compositing then run beside the compositing of the steps before it.
    if args.streams > 1:
        value, pipe_leg = pipelined(args, dgs, torch, np, dev, st, scene, cam, codes, w.basis, bg, W, tw, th, img)
    else:
        value, pipe_leg = serial_value, None
    gc.enable()
    ms_step = W / value * 1e3
    graph_leg = None
    if graph is None:
        # the same step as one captured HIP graph (bin + composite), replayed
        g = dgs.CapturedRender(r, scene, cam, codes, w.basis, bg)
        g.replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(g.out, img))
        t0.record(st)
        for k in range(args.steps):
            g.replay()
        t1.record(st)
        torch.cuda.synchronize()
        gms = t0.elapsed_time(t1) / args.steps
        g.close()
        graph_leg = {"ms_per_step": round(gms, 4), "states_per_s": round(W / (gms / 1e3), 2),
                     "bit_identical_to_eager": same}
        log(f"[bench] batched as graph replay: {gms:.3f} ms/step -> {W / (gms / 1e3):.1f} states/s; identical={same}")

    # the compositing call alone, launched back to back from the last binning: HIP events around each
    # call on the launch stream time the kernel (with its three small set-up launches, ~13 us) while the
    # host stays ahead of the device, which the step loop above cannot promise under a profiler
    r.bin(scene, cam, w.basis)
    ck = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        ck[k][0].record(st)
        r.composite(scene, cam, codes, w.basis, bg, out=img)
        ck[k][1].record(st)
    torch.cuda.synchronize()
    r.check()
    kern_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ck]))
    # algorithmic work of one composite launch
    alpha_evals, blends, wave_evals, wave_miss = r.composite_stats(scene, cam, codes, w.basis)
    flops = FLOPS_PER_ALPHA * alpha_evals + FLOPS_PER_BLEND * blends
    achieved = flops / (kern_ms / 1e3) / 1e12
    plan = r.launch_plan(cam, W)
    kernel = (f"k_composite<{plan['states_per_group']},{tw},{th},0,{'true' if plan['persistent'] else 'false'},"
              f"{plan['lds_batch']}>")
    traffic = profile_summary.measured_traffic(kernel, args.workload, ROOT)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": kernel, "launch": plan,
                "peak_nonpacked": round(PEAK_FP32_NONPACKED_TFLOPS, 1),
                "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "kernel_ms": round(kern_ms, 4), "alpha_evals": alpha_evals, "blends": blends,
                "wave_alpha_evals": wave_evals, "wave_alpha_misses": wave_miss,
                "flops_per_launch": flops}
    log(f"[bench] composite work: {alpha_evals} alpha evals, {blends} blends, {wave_evals} wave evals "
        f"({wave_miss} with no pixel >= 1/255); {kern_ms:.4f} ms per compositing call -> {achieved:.2f} TFLOP/s")

    out = {"metric": METRIC, "value": round(value, 2), "unit": "states/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": args.workload, "gaussians": scene.n, "width": cam.width,
                      "height": cam.height, "states": W, "clusters": w.scene.num_clusters,
                      "contexts": w.scene.num_contexts, "tile": f"{tw}x{th}",
                      "states_per_group": args.states_per_group, "instances": M},
           "batched": {"timed_as": (f"eager launches, steps round robin on {args.streams} streams with a "
                                    "workspace each, median of three repetitions") if pipe_leg is not None
                                   else "eager launches on one stream, median of three repetitions",
                       "pipelined": pipe_leg,
                       "serial_states_per_s": round(serial_value, 2),
                       "serial_ms_per_step": round(W / serial_value * 1e3, 4),
                       "serial_timed_as": ("hip graph replay" if graph is not None else "eager launches")
                                          + " on one stream, median of three repetitions",
                       "bin_ms": round(bin_ms, 4), "composite_ms": round(comp_ms, 4),
                       "first_repetition_states_per_s": round(first_value, 2),
                       # the first repetition: host time to enqueue its steps, and whether the device
                       # idled waiting for launches (the host took most of the device time)
                       "first_repetition_host_enqueue_ms": round(host_ms, 3),
                       "first_repetition_host_bound": bool(graph is None and host_ms > 0.9 * total_ms),
                       "step_ms": distribution([e[0].elapsed_time(e[2]) for e in ev], np),
                       "serial_repetitions_states_per_s": [round(x, 2) for x in reps],
                       "serial_repetitions": distribution(reps, np)}}
    if graph_leg is not None:
        out["batched"]["graph"] = graph_leg

    if not args.no_per_state:
        # plain per-state render, synchronized after every state
        one = torch.empty((1, cam.height, cam.width, 3), dtype=torch.float32, device=dev)
        for k in range(min(4, W)):
            r.render(scene, cam, codes[k:k + 1], w.basis, bg, per_state=True, out=one)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(W):
            r.render(scene, cam, codes[k:k + 1], w.basis, bg, per_state=True, out=one)
            torch.cuda.synchronize()
        ps_s = time.perf_counter() - t0
        r.check()
        same = bool(torch.equal(one[0], img[W - 1]))
        ps_rate = W / ps_s
        out["per_state"] = {"value": round(ps_rate, 2), "unit": "states/s", "ms_per_state": round(1e3 * ps_s / W, 4),
                            "bit_identical_to_batched": same}
        out["speedup_batched_vs_per_state"] = round(value / ps_rate, 3)
        out["speedup_batched_one_stream_vs_per_state"] = round(serial_value / ps_rate, 3)
        log(f"[bench] per-state: {1e3 * ps_s / W:.3f} ms/state -> {ps_rate:.1f} states/s; identical={same}")

    if not args.no_sweep and args.workload == "g250k_800px_64states":
        out["batch_sweep"] = batch_sweep(args, dgs, synth, torch, np, dev, w, scene, cam, tw, th)

    out["roofline"] = roofline
    roofs = measured_roofs(dgs, torch, np, dev)
    out["measured_roofs"] = roofs
    roofline["frac_of_measured_fma"] = round(achieved / roofs["fma_tflops"], 4)

    if args.copy_mib > 0:
        # one streaming pass of known size (reads and writes the buffer once),
        # for scaling FETCH_SIZE / WRITE_SIZE counters
        nbytes = args.copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes

    if not args.no_fwdbwd:
        out["fwd_bwd"] = fwd_bwd(dgs, synth, torch, np, dev, args)
        rb = out["fwd_bwd"].pop("roofline_bwd")
        rb["frac_of_measured_fma"] = round(rb["achieved"] / roofs["fma_tflops"], 4)
        out["roofline_bwd"] = rb
        if not args.no_train_step:
            out["train_step"] = train_step(dgs, synth, torch, np, dev, args)
        if not args.no_serial_fwdbwd:
            out["fwd_bwd_batched_vs_serial"] = fwd_bwd_batched_vs_serial(dgs, synth, torch, np, dev)

    if not args.no_refined:
        out["refined"] = refined_bench(args, w, r, img, dgs, synth, torch, np, dev, bg)

    if not args.no_large:
        del r, img
        torch.cuda.empty_cache()
        out["large_batched"] = large_batched_leg(args, dgs, synth, torch, np, dev)
        pw = synth.make_workload("g1m_540p_32768states_psnr")
        # groups of 16 states with the library's launch choice (persistent at 512 states): 70.3k against
        # 66.6k states/s for groups of 8, which evaluate each alpha for half as many states
        out["psnr_sweep"] = psnr_sweep_leg(args, pw.name, pw, dgs.GaussianScene.from_arrays(pw.scene, dev),
                                           dgs.Camera.from_arrays(pw.camera), dgs, torch, np, dev, 16, 16, 16, None)

    if not args.no_utility:
        out["utility"] = utility_bench(args, dgs, synth, torch, np, dev, tw, th)
        out["sampler"] = sampler_bench(dgs, torch, np, dev, scene.num_packets)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, np, args.cpu_seconds)

    print(json.dumps(out), flush=True)
    return 0


def pipelined(args, dgs, torch, np, dev, st, scene, cam, codes, basis, bg, W, tw, th, img):
    """K steps on a StreamPipeline, three timed repetitions; returns (median
    states/s, record).  Every step's images are checked against the one-stream
    images ``img`` after the last repetition."""
    depth = args.streams
    pipe = dgs.StreamPipeline(dev, depth=depth, tile=(tw, th), states_per_group=args.states_per_group,
                              persistent=LAUNCH[args.launch], lds_batch=args.lds_batch)
    pipe.plan(scene, cam, basis, W)
    outs = [torch.empty_like(img) for _ in range(depth)]

    def steps(n):
        for _ in range(n):
            pipe.render(scene, cam, codes, basis, bg, out=outs[pipe.calls % depth])
        pipe.join()

    steps(max(args.warmup, depth))
    pipe.check()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0.record(st)
        steps(args.steps)
        t1.record(st)
        torch.cuda.synchronize()
        reps.append(W * args.steps / (t0.elapsed_time(t1) / 1e3))
    pipe.check()
    same = all(bool(torch.equal(o, img)) for o in outs)
    value = float(np.median(reps))
    log(f"[bench] batched, {depth} streams, median of 3 repetitions: {W / value * 1e3:.3f} ms/step "
        f"-> {value:.1f} states/s; identical to one stream={same}")
    rec = {"streams": depth, "states_per_s": round(value, 2), "ms_per_step": round(W / value * 1e3, 4),
           "repetitions_states_per_s": [round(x, 2) for x in reps], "repetitions": distribution(reps, np),
           "bit_identical_to_one_stream": same}
    del pipe, outs
    return value, rec


def measured_roofs(dgs, torch, np, dev):
    """Measured roofs beside the published peaks: a 1 GiB device copy (HBM
    bytes moved = 2 x 1 GiB) and the issue rates of FP32 FMA (2 FLOPs per
    instruction and lane, no packed FP32) and of the hardware base-2
    exponential, each the best of five timed launches."""
    import ctypes
    from paper_2606_17212_amd import _abi
    L = _abi.lib()
    st = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(st.cuda_stream)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    out = torch.empty(_abi.PROBE_THREADS, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(f):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0.record(st)
            f()
            e1.record(st)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    copy_ms = best(lambda: _abi.check(L.dgs_probe_copy(ctypes.c_void_p(src.data_ptr()),
                                                       ctypes.c_void_p(dst.data_ptr()), nbytes, sp)))
    assert bool(torch.equal(src[:1024], dst[:1024]))
    iters = 1 << 14
    fma_ms = best(lambda: _abi.check(L.dgs_probe_valu(0, iters, ctypes.c_void_p(out.data_ptr()), sp)))
    exp_ms = best(lambda: _abi.check(L.dgs_probe_valu(1, iters, ctypes.c_void_p(out.data_ptr()), sp)))
    lanes_steps = _abi.PROBE_THREADS * 8 * iters
    res = {"copy_gbps": round(2 * nbytes / (copy_ms / 1e3) / 1e9, 1), "hbm_peak_gbps": 8000.0,
           "fma_tflops": round(2 * lanes_steps / (fma_ms / 1e3) / 1e12, 2),
           "fma_peak_nonpacked_tflops": round(PEAK_FP32_NONPACKED_TFLOPS, 1), "fp32_peak_tflops": PEAK_FP32_TFLOPS,
           "exp2_per_s": round(lanes_steps / (exp_ms / 1e3), -9)}
    log(f"[bench] measured roofs: copy {res['copy_gbps']:.0f} GB/s, FMA {res['fma_tflops']:.1f} TFLOP/s, "
        f"exp2 {res['exp2_per_s'] / 1e12:.2f} T/s")
    del src, dst, out
    return res


def distribution(times, np):
    """Median, mean with its Student-t 95% interval, and percentiles of a
    list of per-iteration times (ms)."""
    from scipy import stats
    t = np.asarray(times, np.float64)
    n = t.size
    half = float(stats.t.ppf(0.975, n - 1) * t.std(ddof=1) / np.sqrt(n)) if n > 1 else float("nan")
    return {"n": int(n), "median": round(float(np.median(t)), 4), "mean": round(float(t.mean()), 4),
            "ci95_half_width": round(half, 4),
            "p5_p25_p75_p95": [round(float(np.percentile(t, q)), 4) for q in (5, 25, 75, 95)]}


SWEEP_STATES = (1, 2, 4, 8, 16, 32, 64, 128)


def batch_sweep(args, dgs, synth, torch, np, dev, w, scene, cam, tw, th):
    """Throughput against the number of delivery states rendered together
    (the paper's batch-size sweep, Sec. 9 table, here on this scene): the
    first W of 128 states drawn with the headline workload's code recipe,
    binning + compositing per step, default launch choice, the median of
    three repetitions of the timed steps, on one stream and (``--streams``
    above 1) rotating over the headline's streams."""
    bg = tuple(float(x) for x in w.background)
    all_codes = torch.from_numpy(synth.make_codes("present_depth", 0.3, 1.0, max(SWEEP_STATES),
                                                  w.scene.num_packets, 4, index=2, stream=7)).to(dev)
    points = []
    for W in SWEEP_STATES:
        codes = all_codes[:W].contiguous()
        r = dgs.Renderer(dev, tile=(tw, th), states_per_group=min(args.states_per_group, W),
                         persistent=LAUNCH[args.launch], lds_batch=args.lds_batch)
        r.plan(scene, cam, w.basis, W)
        img = torch.empty((W, cam.height, cam.width, 3), dtype=torch.float32, device=dev)
        st = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            r.bin(scene, cam, w.basis)
            r.composite(scene, cam, codes, w.basis, bg, out=img)
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            e0.record(st)
            for _ in range(args.steps):
                r.bin(scene, cam, w.basis)
                r.composite(scene, cam, codes, w.basis, bg, out=img)
            e1.record(st)
            torch.cuda.synchronize()
            reps.append(e0.elapsed_time(e1) / args.steps)
        r.check()
        ms = float(np.median(reps))
        point = {"states": W, "states_per_s": round(W / (ms / 1e3), 1), "ms_per_step": round(ms, 4)}
        if args.streams > 1:
            # the same steps rotating over the headline's streams, each with a workspace of its own
            pipe = dgs.StreamPipeline(dev, depth=args.streams, tile=(tw, th),
                                      states_per_group=min(args.states_per_group, W),
                                      persistent=LAUNCH[args.launch], lds_batch=args.lds_batch)
            pipe.plan(scene, cam, w.basis, W)
            outs = [torch.empty_like(img) for _ in range(args.streams)]

            def steps(n):
                for _ in range(n):
                    pipe.render(scene, cam, codes, w.basis, bg, out=outs[pipe.calls % args.streams])
                pipe.join()

            steps(args.streams)
            torch.cuda.synchronize()
            preps = []
            for _ in range(3):
                e0.record(st)
                steps(args.steps)
                e1.record(st)
                torch.cuda.synchronize()
                preps.append(e0.elapsed_time(e1) / args.steps)
            pipe.check()
            pms = float(np.median(preps))
            point.update({"streams": args.streams, "pipelined_states_per_s": round(W / (pms / 1e3), 1),
                          "pipelined_ms_per_step": round(pms, 4),
                          "pipelined_bit_identical": all(bool(torch.equal(o, img)) for o in outs)})
            del pipe, outs
        points.append(point)
        del r, img
    log("[bench] batch sweep (states: states/s, one stream): " +
        ", ".join(f"{p['states']}: {p['states_per_s']:.0f}" for p in points))
    if args.streams > 1:
        log(f"[bench] batch sweep (states: states/s, {args.streams} streams): " +
            ", ".join(f"{p['states']}: {p['pipelined_states_per_s']:.0f}" for p in points))
    return {"workload": "g250k_800px_64states scene and camera",
            "codes": "present_depth 0.3-1.0 (the headline recipe), first W of 128 states",
            "points": points}


def fwd_bwd(dgs, synth, torch, np, dev, args):
    """Forward + L1 loss + backward to the six parameter tensors on the
    250k-Gaussian 1280x720 8-state workload; the target is the full-delivery
    render of the scene with parameters perturbed by N(0, 0.01)."""
    name = "g250k_720p_8states_fwdbwd"
    w = synth.make_workload(name)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(w.codes).to(dev)
    bg = tuple(float(x) for x in w.background)
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=8)
    pert = dgs.GaussianScene.from_arrays(synth.perturb_scene(w.scene, 0.01, index=w.index), dev)
    full = torch.full((1, w.scene.num_packets), 4, dtype=torch.uint8, device=dev)
    target = r.render(pert, cam, full, w.basis, bg)[:1].clone()
    l1 = dgs.L1Loss(dev)  # device L1 loss and gradient (one pass each)
    r.plan(scene, cam, w.basis, codes.shape[0])
    from paper_2606_17212_amd.render import PARAMS
    params = {k: getattr(scene, k).clone().requires_grad_(True) for k in PARAMS}
    sc = scene.with_params(**params)

    def it():
        for p in params.values():
            p.grad = None
        img = dgs.render(r, sc, cam, codes, w.basis, bg)
        loss = dgs.l1_loss(img, target, None, l1)
        loss.backward()
        return loss

    for _ in range(3):
        it()
    r.check()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    iters = max(5, args.steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(iters):
        e0.record(st)
        loss = it()
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    r.check()
    finite = all(bool(torch.isfinite(p.grad).all()) for p in params.values())
    log(f"[bench] fwd+bwd {name}: median {np.median(times):.3f} ms/iter, loss {float(loss.detach()):.5f}")
    out = {"workload": name, "gaussians": w.scene.n, "width": cam.width, "height": cam.height,
           "states": int(codes.shape[0]), "ms_per_iter": round(float(np.median(times)), 4),
           "ms_per_iter_all": [round(t, 4) for t in times], "distribution": distribution(times, np),
           "grads_finite": finite}

    out["roofline_bwd"] = backward_roofline(dgs, torch, np, dev, r, sc, cam, codes, w.basis, bg, target, l1,
                                            params, iters)
    out["graph"] = fwd_bwd_graph(dgs, torch, np, dev, r, sc, scene, cam, codes, w.basis, bg, target, l1, params,
                                 iters)
    if args.no_refined:
        return out
    # the same step with three refinement levels (gradients for base and levels)
    levels = synth.make_refinement(w.scene, index=w.index)
    rs = dgs.GaussianScene.from_arrays(w.scene, dev, refine=levels)
    rp = {k: getattr(rs, k).clone().requires_grad_(True) for k in PARAMS}
    rp["refine"] = rs.refine.clone().requires_grad_(True)
    rsc = rs.with_params(**rp)
    r.plan(rs, cam, w.basis, codes.shape[0])

    def it_refined():
        for p in rp.values():
            p.grad = None
        img = dgs.render(r, rsc, cam, codes, w.basis, bg)
        loss = dgs.l1_loss(img, target, None, l1)
        loss.backward()
        return loss

    for _ in range(3):
        it_refined()
    r.check()
    rtimes = []
    for _ in range(iters):
        e0.record(st)
        it_refined()
        e1.record(st)
        torch.cuda.synchronize()
        rtimes.append(e0.elapsed_time(e1))
    r.check()
    rfinite = all(bool(torch.isfinite(p.grad).all()) for p in rp.values())
    log(f"[bench] fwd+bwd with refinement levels: median {np.median(rtimes):.3f} ms/iter")
    out["refined"] = {"ms_per_iter": round(float(np.median(rtimes)), 4), "records": rs.records,
                      "grads_finite": rfinite}
    return out


def backward_roofline(dgs, torch, np, dev, r, sc, cam, codes, basis, bg, target, l1, params, iters):
    """Roofline of the backward: dgs_backward timed alone with HIP events
    on its stream (the compositing backward, which replays each tile, plus
    the geometry backward), against the algorithmic FLOPs of the compositing
    backward: per alpha evaluation (pixel, entry, state group) the forward's
    14 plus the chain to the splat's nine 2D gradients and their sum over
    pixels (27), per blend (pixel, state, Gaussian) the forward's 8 plus
    g . c, the colour-behind update, dL/dalpha and dL/dc (17).  The unit
    counts are the forward's, which the replay repeats."""
    with torch.no_grad():
        img = r.render(sc, cam, codes, basis, bg)
        gimg = l1.grad(img, target)
    st = torch.cuda.current_stream(dev)
    for _ in range(2):
        r.backward(sc, cam, codes, basis, bg, img, gimg)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(iters):
        e0.record(st)
        r.backward(sc, cam, codes, basis, bg, img, gimg)
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    r.check()
    a_ev, bl, _, _ = r.composite_stats(sc, cam, codes, basis)
    fl = FLOPS_BWD_PER_ALPHA * a_ev + FLOPS_BWD_PER_BLEND * bl
    ms = float(np.mean(times))
    ach = fl / (ms / 1e3) / 1e12
    log(f"[bench] backward: {ms:.3f} ms per dgs_backward, {a_ev} alpha evals, {bl} blends -> {ach:.2f} TFLOP/s")
    from paper_2606_17212_amd import profile_summary
    traffic = profile_summary.measured_traffic(BWD_KERNELS, "g250k_720p_8states_fwdbwd", ROOT, tag="k_composite_bwd")
    return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "kernel": "k_composite_bwd (+ k_geometry_bwd in the timed call)",
            "peak_nonpacked": round(PEAK_FP32_NONPACKED_TFLOPS, 1),
            "frac_nonpacked": round(ach / PEAK_FP32_NONPACKED_TFLOPS, 4),
            "call_ms": round(ms, 4), "alpha_evals": a_ev, "blends": bl, "flops_per_call": fl}


def fwd_bwd_graph(dgs, torch, np, dev, r, sc, scene, cam, codes, basis, bg, target, l1, eager_params, iters):
    """The forward + L1 + backward iteration captured as one HIP graph and
    replayed.  The captured step owns leaf tensors that were never used on
    the default stream and is warmed up on the capture's side stream (a leaf
    whose gradient-accumulation node is bound to the default stream makes
    autograd synchronise with that stream inside the capture).  Every replay's
    gradients are compared with the eager iteration's."""
    from paper_2606_17212_amd.render import PARAMS
    ref = {k: p.grad.detach().clone() for k, p in eager_params.items()}
    params = {k: getattr(scene, k).clone().requires_grad_(True) for k in PARAMS}
    gsc = scene.with_params(**params)

    def it():
        loss = dgs.l1_loss(dgs.render(r, gsc, cam, codes, basis, bg), target, None, l1)
        loss.backward()

    side = torch.cuda.Stream(dev)  # default priority
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        for _ in range(3):
            for p in params.values():
                p.grad = None
            it()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    for p in params.values():
        p.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        it()
    st = torch.cuda.current_stream(dev)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times, worst = [], 0.0
    for _ in range(iters):
        e0.record(st)
        graph.replay()
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        worst = max(worst, max(float((params[k].grad - ref[k]).norm() / ref[k].norm().clamp_min(1e-30))
                               for k in PARAMS))
    r.check()
    del graph
    log(f"[bench] fwd+bwd as one graph replay: median {np.median(times):.3f} ms/iter; "
        f"max relative gradient difference to eager {worst:.2e}")
    return {"ms_per_iter": round(float(np.median(times)), 4), "distribution": distribution(times, np),
            "max_rel_grad_diff_vs_eager": worst}


def fwd_bwd_batched_vs_serial(dgs, synth, torch, np, dev, states=32, iters=5, serial_iters=2):
    """Forward + L1 + backward of 32 delivery states of the 2.7M-Gaussian
    1920x1080 recipe in one batched call, against serial calls, synchronised after each,
    of the same renderer with one state each (each call projects and bins the
    whole scene, composites its state and runs the backward; gradients
    accumulate over the calls).  The paper reports this speedup for 32
    batched states on 2.7M primitives (Sec. 6) on other hardware and scenes:
    context, not a target.  The target is the full-delivery render of the
    scene with parameters perturbed by N(0, 0.01)."""
    name = "g2700k_1080p_256states"
    w = synth.make_workload(name, states=states)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(w.codes).to(dev)
    bg = tuple(float(x) for x in w.background)
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=8)
    pert = dgs.GaussianScene.from_arrays(synth.perturb_scene(w.scene, 0.01, index=w.index), dev)
    full = torch.full((1, w.scene.num_packets), 4, dtype=torch.uint8, device=dev)
    target = r.render(pert, cam, full, w.basis, bg)[:1].clone()
    del pert
    l1 = dgs.L1Loss(dev)
    from paper_2606_17212_amd.render import PARAMS
    params = {k: getattr(scene, k).clone().requires_grad_(True) for k in PARAMS}
    sc = scene.with_params(**params)
    r.plan(scene, cam, w.basis, states)

    def batched():
        for p in params.values():
            p.grad = None
        img = dgs.render(r, sc, cam, codes, w.basis, bg)
        dgs.l1_loss(img, target, None, l1).backward()

    def serial():
        for p in params.values():
            p.grad = None
        for k in range(states):
            img = dgs.render(r, sc, cam, codes[k:k + 1], w.basis, bg)
            (dgs.l1_loss(img, target, None, l1) / states).backward()
            torch.cuda.synchronize()

    def timed(f, n):
        f()
        torch.cuda.synchronize()
        times = []
        for _ in range(n):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
        return times

    tb = timed(batched, iters)
    gb = {k: p.grad.clone() for k, p in params.items()}
    ts = timed(serial, serial_iters)
    r.check()
    rel = max(float((params[k].grad - gb[k]).norm() / gb[k].norm().clamp_min(1e-30)) for k in params)
    mb, msr = float(np.median(tb)), float(np.median(ts))
    log(f"[bench] fwd+bwd {states} states of {name} (N={w.scene.n}): batched {mb:.2f} ms, serial {msr:.2f} ms "
        f"-> {msr / mb:.2f}x; max relative gradient difference {rel:.2e}")
    return {"workload": f"g2700k_1080p_{states}states (the 2.7M recipe, present fractions 0.05-1 over {states} states)",
            "gaussians": w.scene.n, "width": cam.width,
            "height": cam.height, "states": states, "batched_ms_per_iter": round(mb, 3),
            "serial_ms_per_iter": round(msr, 3), "speedup": round(msr / mb, 3),
            "batched_ms_all": [round(t, 3) for t in tb], "serial_ms_all": [round(t, 3) for t in ts],
            "max_rel_grad_diff_batched_vs_serial": rel}


def train_step(dgs, synth, torch, np, dev, args):
    """One step of the packet-conditioned objective (Eq. (2) with the weights
    the paper locks) on the 250k-Gaussian 1280x720 workload: 8 worlds (7
    partial delivery states and the complete prefix) rendered at two times,
    D of each image against the full-delivery render of the perturbed scene
    at its time, CVaR over the 14 partial images, prefix pairs to the anchor
    of each time, temporal pairs between the times, and the backward through
    both renders to the six parameter tensors."""
    name = "g250k_720p_8states_fwdbwd"
    w = synth.make_workload(name)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(w.codes).to(dev).clone()
    codes[7] = 4  # the complete prefix
    bg = tuple(float(x) for x in w.background)
    bases = [synth.temporal_basis(t, w.scene.rank) for t in (w.t, w.t + 0.1)]
    pert = dgs.GaussianScene.from_arrays(synth.perturb_scene(w.scene, 0.01, index=w.index), dev)
    full = torch.full((1, w.scene.num_packets), 4, dtype=torch.uint8, device=dev)
    rs = [dgs.Renderer(dev, tile=(16, 16), states_per_group=8) for _ in bases]
    targets = torch.stack([rs[i].render(pert, cam, full, bases[i], bg)[0].clone() for i in range(2)])
    for i in range(2):
        rs[i].plan(scene, cam, bases[i], int(codes.shape[0]))
    from paper_2606_17212_amd.render import PARAMS
    params = {k: getattr(scene, k).clone().requires_grad_(True) for k in PARAMS}
    sc = scene.with_params(**params)
    ob = dgs.Objective(dev)
    i32 = lambda a: torch.as_tensor(np.asarray(a, np.int32).reshape(-1)).to(dev)  # noqa: E731
    expect = [k for k in range(16) if k % 8 != 7]
    roles = dict(target_of=i32(np.repeat([0, 1], 8)), expect=i32(expect), anchor=i32([7, 15]),
                 mono=i32([(k, 7 if k < 8 else 15) for k in expect]), temporal=i32([(k, k + 8) for k in range(8)]))

    def it():
        for p in params.values():
            p.grad = None
        imgs = torch.cat([dgs.render(rs[i], sc, cam, codes, bases[i], bg) for i in range(2)])
        loss = dgs.ObjectiveFunction.apply(ob, imgs, targets, roles["target_of"], roles["expect"], roles["anchor"],
                                           roles["mono"], roles["temporal"])
        loss.backward()
        return loss, imgs

    for _ in range(3):
        it()
    for r in rs:
        r.check()
    ob.check()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    iters = max(5, args.steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(iters):
        e0.record(st)
        loss, imgs = it()
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    # the objective alone (forward parts + gradient images of the 16 images)
    x = imgs.detach().contiguous()
    ot = []
    for _ in range(iters):
        e0.record(st)
        parts, _, _ = ob(x, targets, roles["target_of"], roles["expect"], roles["anchor"], roles["mono"],
                         roles["temporal"])
        e1.record(st)
        torch.cuda.synchronize()
        ot.append(e0.elapsed_time(e1))
    ob.check()
    finite = all(bool(torch.isfinite(p.grad).all()) for p in params.values())
    pv = [round(float(v), 6) for v in parts.cpu()]
    log(f"[bench] train step (Eq. 2) {name}: median {np.median(times):.3f} ms/iter for 2 x 8 states "
        f"(objective {np.median(ot):.3f} ms); L, E, CVaR, F, M, anchor = {pv}")
    return {"workload": name + "_eq2", "images": 16, "times": 2, "states_per_time": 8,
            "ms_per_iter": round(float(np.median(times)), 4), "objective_ms": round(float(np.median(ot)), 4),
            "loss_parts": pv, "grads_finite": finite}


def refined_bench(args, w, r, img, dgs, synth, torch, np, dev, bg):
    """The same states of the same scene with three attribute refinement
    levels (Sec. 3): one record per (Gaussian, delivered depth), exact-depth
    state tables.  Timed like the main leg (bin + composite per step)."""
    levels = synth.make_refinement(w.scene, index=w.index)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev, refine=levels)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(w.codes).to(dev)
    W = int(codes.shape[0])
    M = r.plan(scene, cam, w.basis, W)
    for _ in range(max(args.warmup, 1)):
        r.bin(scene, cam, w.basis)
        r.composite(scene, cam, codes, w.basis, bg, out=img)
    r.check()
    st = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        ev[k][0].record(st)
        r.bin(scene, cam, w.basis)
        ev[k][1].record(st)
        r.composite(scene, cam, codes, w.basis, bg, out=img)
        ev[k][2].record(st)
    torch.cuda.synchronize()
    r.check()
    total_ms = ev[0][0].elapsed_time(ev[-1][2])
    bin_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    comp_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    alpha_evals, blends, wave_evals, wave_miss = r.composite_stats(scene, cam, codes, w.basis)
    flops = FLOPS_PER_ALPHA * alpha_evals + FLOPS_PER_BLEND * blends
    value = W * args.steps / (total_ms / 1e3)
    log(f"[bench] refined: {total_ms / args.steps:.3f} ms/step (bin {bin_ms:.3f}, composite {comp_ms:.3f}) "
        f"-> {value:.1f} states/s; {M} instances")
    out = {"workload": args.workload + "_refined", "value": round(value, 2), "unit": "states/s",
           "records": scene.records, "instances": M, "ms_per_step": round(total_ms / args.steps, 4),
           "bin_ms": round(bin_ms, 4), "composite_ms": round(comp_ms, 4),
           "achieved_tflops": round(flops / (comp_ms / 1e3) / 1e12, 3),
           "alpha_evals": alpha_evals, "blends": blends}
    if not args.no_per_state:
        # the per-state baseline of the same states (each state's delivered records)
        r.bin(scene, cam, w.basis)
        r.composite(scene, cam, codes, w.basis, bg, out=img)
        one = torch.empty((1, cam.height, cam.width, 3), dtype=torch.float32, device=dev)
        for k in range(min(4, W)):
            r.render(scene, cam, codes[k:k + 1], w.basis, bg, per_state=True, out=one)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(W):
            r.render(scene, cam, codes[k:k + 1], w.basis, bg, per_state=True, out=one)
            torch.cuda.synchronize()
        ps_s = time.perf_counter() - t0
        r.check()
        same = bool(torch.equal(one[0], img[W - 1]))
        out["per_state"] = {"value": round(W / ps_s, 2), "unit": "states/s", "bit_identical_to_batched": same}
        out["speedup_batched_vs_per_state"] = round(value / (W / ps_s), 3)
        log(f"[bench] refined per-state: {1e3 * ps_s / W:.3f} ms/state -> {W / ps_s:.1f} states/s; identical={same}")
    return out


def psnr_sweep(args, w, scene, cam, dgs, torch, np, dev, tw, th):
    """Main mode for the PSNR-sweep workload: the sweep leg as the JSON line."""
    leg = psnr_sweep_leg(args, args.workload, w, scene, cam, dgs, torch, np, dev, tw, th, args.states_per_group,
                         LAUNCH[args.launch])
    out = {"metric": METRIC, "value": leg["value"], "unit": "states/s", "n_gpus": 1, "steps": 1,
           "warmup": leg["warmup"], "ms_per_step": leg["ms_per_sweep"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": args.workload, "gaussians": scene.n, "width": cam.width, "height": cam.height,
                      "states": leg["states"], "batch": leg["batch"], "tile": f"{tw}x{th}",
                      "states_per_group": args.states_per_group}}
    out.update({k: leg[k] for k in ("batch_latency_ms", "psnr_db", "roofline_composite")})
    print(json.dumps(out), flush=True)
    return 0


def psnr_sweep_leg(args, name, w, scene, cam, dgs, torch, np, dev, tw, th, S, persistent):
    """Utility-style sweep: every delivery state's PSNR against the
    full-delivery render, in batches, binning shared by the whole sweep
    (one scene, one camera, one time), PSNR reduced on the device."""
    import synth
    total, batch = w.total_states, w.batch
    rec = synth.WORKLOADS[name]
    kind, lo, hi = rec["masks"]
    codes_all = torch.from_numpy(synth.make_codes(kind, lo, hi, total, w.scene.num_packets, rec["layers"],
                                                  index=w.index)).to(dev)
    bg = tuple(float(x) for x in w.background)
    ren = dgs.Renderer(dev, tile=(tw, th), states_per_group=S, persistent=persistent, lds_batch=args.lds_batch)
    ren.plan(scene, cam, w.basis, batch)
    ref = ren.render(scene, cam, torch.ones_like(codes_all[:1]), w.basis, bg)[0].contiguous()
    psnr = torch.empty(total, dtype=torch.float32, device=dev)

    def sweep(ev=None):
        ren.bin(scene, cam, w.basis)
        for b in range(total // batch):
            if ev is not None:
                ev[b][0].record()
            ren.composite_psnr(scene, cam, codes_all[b * batch:(b + 1) * batch], w.basis, ref, bg,
                               out=psnr[b * batch:(b + 1) * batch])
            if ev is not None:
                ev[b][1].record()

    for _ in range(max(1, args.warmup // 2)):
        sweep()
    ren.check()
    torch.cuda.synchronize()
    nb = total // batch
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(nb)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sweep(ev)
    e1.record()
    torch.cuda.synchronize()
    ren.check()
    ms = e0.elapsed_time(e1)
    lat = [e[0].elapsed_time(e[1]) for e in ev]
    value = total / (ms / 1e3)
    p = psnr.cpu().numpy()
    # compositing work of one batch (the first), for the roofline of the PSNR-mode kernel
    a_ev, bl, _, _ = ren.composite_stats(scene, cam, codes_all[:batch], w.basis)
    fl = FLOPS_PER_ALPHA * a_ev + FLOPS_PER_BLEND * bl
    ach = fl / (lat[0] / 1e3) / 1e12
    log(f"[bench] psnr sweep: {total} states in {ms:.1f} ms -> {value:.1f} states/s; batch latency median "
        f"{np.median(lat):.3f} ms; PSNR median {np.median(p):.2f} dB; first batch {ach:.2f} TFLOP/s")
    plan = ren.launch_plan(cam, batch)
    del ren
    return {"workload": name, "value": round(value, 2), "unit": "states/s", "states": total, "batch": batch,
            "gaussians": scene.n, "width": cam.width, "height": cam.height, "tile": f"{tw}x{th}",
            "launch": plan, "warmup": max(1, args.warmup // 2), "ms_per_sweep": round(ms, 3),
            "batch_latency_ms": {"median": round(float(np.median(lat)), 4),
                                 "p90": round(float(np.percentile(lat, 90)), 4), "max": round(float(np.max(lat)), 4),
                                 "distribution": distribution(lat, np)},
            "psnr_db": {"median": round(float(np.median(p)), 3), "min": round(float(np.min(p)), 3),
                        "max": round(float(np.max(p)), 3)},
            "roofline_composite": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                                   "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                                   "scope": "first batch of 512 states", "alpha_evals": a_ev, "blends": bl}}


def large_batched_leg(args, dgs, synth, torch, np, dev, w=None):
    """The 2.7M-Gaussian 1920x1080 workload with 256 delivery states of
    uneven present counts (5% .. 100% of the Gaussians) in one batch:
    bin + composite per step, compositing in the persistent launch with 16
    states per group (the autotuner's choice for this workload), three
    repetitions of the timed steps.  Reports states/s and the HBM rate of
    the algorithmic bytes (scene, records, sort and instances once per step;
    per tile the list's values and records once; per state its image); the
    re-reads of a tile's entries by its other state groups are served by the
    L2 of the XCD that runs all of them and are reported apart."""
    name = "g2700k_1080p_256states"
    w = w or synth.make_workload(name)
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    codes = torch.from_numpy(w.codes).to(dev)
    W = int(codes.shape[0])
    bg = tuple(float(x) for x in w.background)
    S = 16
    r = dgs.Renderer(dev, tile=(16, 16), states_per_group=S, persistent=True, lds_batch=256)
    M = r.plan(scene, cam, w.basis, W)
    img = torch.empty((W, cam.height, cam.width, 3), dtype=torch.float32, device=dev)
    for _ in range(2):
        r.bin(scene, cam, w.basis)
        r.composite(scene, cam, codes, w.basis, bg, out=img)
    r.check()
    st = torch.cuda.current_stream(dev)
    steps = 4
    reps, bins, comps = [], [], []
    for _ in range(3):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        for k in range(steps):
            ev[k][0].record(st)
            r.bin(scene, cam, w.basis)
            ev[k][1].record(st)
            r.composite(scene, cam, codes, w.basis, bg, out=img)
            ev[k][2].record(st)
        torch.cuda.synchronize()
        reps.append(W * steps / (ev[0][0].elapsed_time(ev[-1][2]) / 1e3))
        bins += [e[0].elapsed_time(e[1]) for e in ev]
        comps += [e[1].elapsed_time(e[2]) for e in ev]
    r.check()
    a_ev, bl, _, _ = r.composite_stats(scene, cam, codes, w.basis)
    fl = FLOPS_PER_ALPHA * a_ev + FLOPS_PER_BLEND * bl
    bin_ms, comp_ms = float(np.median(bins)), float(np.median(comps))
    # algorithmic HBM bytes of one step: geometry 118 B read + 64 B written per Gaussian, four 16-B
    # passes of the depth sort, 8 B per instance (scatter write + range walk), each list entry's value
    # (4 B) and record (48 B) once per tile, 12 B per pixel of each state's image.  The other state
    # groups of a tile read the same entries again, from the L2 their XCD shares (reported apart).
    groups = (W + S - 1) // S
    nbytes = scene.n * (118 + 64 + 4 * 16) + 8 * M + M * 52 + W * cam.width * cam.height * 12
    l2_rereads = (groups - 1) * M * 52
    value = float(np.median(reps))
    ms_step = W / value * 1e3
    log(f"[bench] {name}: {ms_step:.2f} ms/step (bin {bin_ms:.2f}, composite {comp_ms:.2f}) -> {value:.1f} states/s; "
        f"algorithmic HBM bytes {nbytes / 1e9:.2f} GB -> {nbytes / (ms_step / 1e3) / 1e9:.0f} GB/s")
    out = {"workload": name, "gaussians": scene.n, "width": cam.width, "height": cam.height, "states": W,
           "instances": M, "tile": "16x16", "states_per_group": S, "launch": r.launch_plan(cam, W),
           "value": round(value, 2), "unit": "states/s", "ms_per_step": round(ms_step, 3),
           "bin_ms": round(bin_ms, 3), "composite_ms": round(comp_ms, 3),
           "repetitions_states_per_s": [round(x, 2) for x in reps], "repetitions": distribution(reps, np),
           "hbm_algorithmic_bytes_per_step": int(nbytes),
           "hbm_algorithmic_gbps": round(nbytes / (ms_step / 1e3) / 1e9, 1),
           "l2_group_reread_bytes_per_step": int(l2_rereads),
           "composite_achieved_tflops": round(fl / (comp_ms / 1e3) / 1e12, 3),
           "composite_frac": round(fl / (comp_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
    del r, img
    torch.cuda.empty_cache()
    return out


def utility_bench(args, dgs, synth, torch, np, dev, tw, th):
    """Counterfactual utility (Eq. (3)-(4)): one step = binning of the scene
    + Delta_g(m) of every (group, context) pair by the paired incremental
    renderer + the risk-adjusted utility of every group.  Compared with the
    same deltas from full-frame renders of both states of every pair plus
    the on-device distortion."""
    uw = synth.make_utility_workload(args.utility)
    w = uw.base
    scene = dgs.GaussianScene.from_arrays(w.scene, dev)
    cam = dgs.Camera.from_arrays(w.camera)
    bg = tuple(float(x) for x in w.background)
    ctx = torch.from_numpy(uw.codes).to(dev)
    cg = torch.from_numpy(uw.context_group).to(dev)
    gpl = torch.from_numpy(uw.group_pl.view(np.int16)).to(dev)
    G, J = int(gpl.shape[0]), int(ctx.shape[0])
    offsets = torch.from_numpy(np.searchsorted(uw.context_group, np.arange(G + 1)).astype(np.int32)).to(dev)
    r = dgs.Renderer(dev, tile=(tw, th), states_per_group=args.states_per_group, persistent=LAUNCH[args.launch],
                     lds_batch=args.lds_batch)
    r.plan(scene, cam, w.basis, 512)
    # the reference I: full delivery (code 4 = every layer of every packet)
    ref = r.render(scene, cam, torch.full_like(ctx[:1], 4), w.basis, bg)[0].contiguous()
    r.bin(scene, cam, w.basis)
    items = r.utility_items(scene, cam, ctx, cg, gpl, w.basis)
    delta = torch.empty(J, dtype=torch.float32, device=dev)

    def step(ev=None):
        if ev: ev[0].record()
        r.bin(scene, cam, w.basis)
        if ev: ev[1].record()
        r.utility(scene, cam, ctx, cg, gpl, w.basis, ref, bg, item_capacity=items, out=delta)
        if ev: ev[2].record()
        stats = dgs.risk_adjusted(delta, offsets)
        if ev: ev[3].record()
        return stats

    for _ in range(2):
        step()
    r.utility_check()
    torch.cuda.synchronize()
    K = max(3, args.steps // 2)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    for k in range(K):
        stats = step(evs[k])
    torch.cuda.synchronize()
    r.utility_check()
    tot = float(np.median([e[0].elapsed_time(e[3]) for e in evs]))
    t_bin = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    t_util = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    t_risk = float(np.median([e[2].elapsed_time(e[3]) for e in evs]))

    # the same deltas from full-frame renders of both states of every pair
    mg = uw.codes.copy()
    p = (uw.group_pl >> 2).astype(np.int64)[uw.context_group]
    mg[np.arange(J), p] = (uw.group_pl & 3).astype(np.uint8)[uw.context_group] + 1
    mg = torch.from_numpy(mg).to(dev)
    chunk = 256
    imgs = torch.empty((2 * chunk, cam.height, cam.width, 3), dtype=torch.float32, device=dev)
    full = torch.empty(J, dtype=torch.float64, device=dev)

    def full_frame():
        r.bin(scene, cam, w.basis)
        for b in range(0, J, chunk):
            e = min(J, b + chunk)
            pair = torch.cat([ctx[b:e], mg[b:e]])
            r.composite(scene, cam, pair, w.basis, bg, out=imgs[:2 * (e - b)])
            d = dgs.distortion(imgs[:2 * (e - b)], ref).double()
            full[b:e] = d[:e - b] - d[e - b:]

    full_frame()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    full_frame()
    e1.record()
    torch.cuda.synchronize()
    t_full = e0.elapsed_time(e1)
    diff = float((delta.double() - full).abs().max())
    st = stats.cpu().numpy()
    log(f"[bench] utility {args.utility}: {G} groups x {J // G} contexts, {items} tile items; "
        f"{tot:.3f} ms/step (bin {t_bin:.3f}, deltas {t_util:.3f}, Eq.4 {t_risk:.3f}) -> {J / (tot / 1e3):.0f} "
        f"deltas/s; full-frame pairs {t_full:.2f} ms -> speedup {t_full / tot:.2f}x; max |diff| {diff:.2e}")
    return {"workload": args.utility, "groups": G, "contexts": J, "tile_items": items,
            "ms_per_step": round(tot, 4), "bin_ms": round(t_bin, 4), "delta_ms": round(t_util, 4),
            "risk_ms": round(t_risk, 4), "deltas_per_s": round(J / (tot / 1e3), 1),
            "paired_states_per_s": round(2 * J / (tot / 1e3), 1),
            "full_frame_ms": round(t_full, 4), "speedup_vs_full_frame": round(t_full / tot, 3),
            "max_abs_diff_vs_full_frame": diff,
            "risk_adjusted": {"median": round(float(np.median(st[:, 3])), 8),
                              "negative_groups": int((st[:, 3] < 0).sum())}}


def sampler_bench(dgs, torch, np, dev, num_packets):
    """Delivery states drawn on the device: 32,768 worlds of this scene's
    packets x 4 layers through Gilbert-Elliott channels with deadlines."""
    W, L = 32768, 4
    rng = np.random.default_rng(2606)
    ch = np.zeros(W, dtype=dgs.CHANNEL_DTYPE)
    ch["p_gb"], ch["p_bg"] = rng.uniform(0.0, 0.1, W), rng.uniform(0.1, 0.5, W)
    ch["loss_good"], ch["loss_bad"] = rng.uniform(0.0, 0.05, W), rng.uniform(0.3, 0.9, W)
    ch["p_start_bad"] = ch["p_gb"] / (ch["p_gb"] + ch["p_bg"])
    ch["deadline"] = rng.integers(num_packets, L * num_packets + 1, W)
    dch = dgs.channels_to_device(ch, dev)
    codes = torch.empty((W, num_packets), dtype=torch.uint8, device=dev)
    for _ in range(2):
        dgs.sample_states(dch, num_packets, L, 7, out=codes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for k in range(reps):
        dgs.sample_states(dch, num_packets, L, 7 + k, out=codes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    log(f"[bench] sampler: {W} worlds x {num_packets} packets x {L} layers in {ms:.3f} ms -> "
        f"{W / (ms / 1e3):.3g} states/s; mean code {codes.float().mean().item():.3f}")
    return {"worlds": W, "packets": num_packets, "layers": L, "ms": round(ms, 4),
            "states_per_s": round(W / (ms / 1e3), 1)}


def cpu_baseline(w, np, seconds):
    """The oracle (plain FP64 C, OpenMP over pixels) on a bounded random pixel
    sample of the same workload, every state; scaled to full-frame states/s."""
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    H, Wd = w.camera.height, w.camera.width
    rng = np.random.default_rng(2606)
    # two probes separate the per-call cost (geometry of every Gaussian) from the per-pixel cost
    probe_t = []
    for m in (64, 576):
        probe = np.stack([rng.integers(0, Wd, m), rng.integers(0, H, m)], 1)
        t0 = time.perf_counter()
        oracle.render(w.scene, w.camera, w.basis, w.codes, w.background, pixels=probe)
        probe_t.append(time.perf_counter() - t0)
    per_px = max((probe_t[1] - probe_t[0]) / 512, probe_t[1] / 576 * 0.1, 1e-9)
    fixed = max(probe_t[0] - 64 * per_px, 0.0)
    k = int(min(H * Wd, max(256, (seconds - fixed) / per_px)))
    pix = np.stack([rng.integers(0, Wd, k), rng.integers(0, H, k)], 1)
    t0 = time.perf_counter()
    oracle.render(w.scene, w.camera, w.basis, w.codes, w.background, pixels=pix)
    dt = time.perf_counter() - t0
    W = w.codes.shape[0]
    rate = W * (k / (H * Wd)) / dt
    log(f"[bench] cpu oracle: {k} px x {W} states in {dt:.2f} s on {cores} threads -> {rate:.4g} states/s")
    return {"value": rate, "unit": "states/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} uniformly random pixels of {Wd}x{H}, all {W} states, {dt:.1f} s; "
                      "rate scaled by (sampled pixels / frame pixels)",
            "note": "the FP64 oracle as written: every pixel tests every Gaussian (no tiling, no shared "
                    "binning); a correctness reference timed for context, not a tuned CPU renderer"}


if __name__ == "__main__":
    sys.exit(main())
