"""Benchmark: filter-bank dataflow graph on one MI355X.

Step = one batched firing of the plain graph SOURCE -> FILTERBANK -> SINK
(with its CONFIG actor) over one batch of frames: control-token production
and decoding, FIFO bookkeeping, the persistent filter-bank launch and the
history update, replayed as a hipGraph.  Inputs (frames written in place in
the source FIFO, side-information in the configuration actor's device queue)
are resident in HBM before the timed region.

Default workload: 4096 frames x 16384 complex64 samples on one stream,
K ~ U{1..10} active branches per frame from control tokens, L = 32 taps,
fp32 arithmetic.  Prints one JSON line.
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

PEAK_FP32_VECTOR_TFLOPS = 157.3     # 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 flop x 2.4 GHz
PEAK_FP32_MATRIX_TFLOPS = 157.3     # 256 CU x 4 SIMD x 2048 flop per 32-cycle 16x16x4 MFMA x 2.4 GHz
PEAK_HBM_GBPS = 8000.0
METRIC = "actor Msamples/s fwd and fwd+bwd, batched vs per-frame, at ≤2e-5 rel err"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    # A freshly started process runs its first couple of dozen full-size
    # forward launches slower: the kernel's cycle count stays the same while
    # the shader clock climbs (per-dispatch GRBM_GUI_ACTIVE), so the default
    # warm-up covers that ramp before either launch mode is timed.
    p.add_argument("--warmup", type=int, default=30)
    p.add_argument("--frames", type=int, default=0, help="override frames per batch (parity/debug)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-per-frame", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--only-c2", action="store_true", help="skip the other workloads")
    p.add_argument("--only", default="", help="run one secondary workload only: c1, c3, c4, c4fit, c5, c5bwd, c2u, paper, host, motion, perframe")
    p.add_argument("--ceilings", action="store_true",
                   help="only the ceiling probes (copy bandwidth, unpacked fp32 FMA, fp32 MFMA)")
    p.add_argument("--copy-calib", action="store_true",
                   help="only copy a 1 GiB buffer twice (HBM counter calibration)")
    p.add_argument("--profile-only", action="store_true",
                   help="only the timed batched steps (for profiler runs)")
    p.add_argument("--fb-variant", default="",
                   help="force this forward kernel variant by name instead of autotuning (profiler runs "
                        "that must see the same kernel in every counter pass)")
    return p.parse_args()


def measured_traffic(kernel_src, record):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    try:
        kv = dict(l.strip().split("=", 1) for l in open(record) if "=" in l)
        h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
        return float(kv["traffic_bytes"]) if kv.get("source_sha256_16") == h else None
    except OSError:
        return None


def measure_ceilings(sweep=False):
    """The device's sustained copy bandwidth, unpacked fp32 FMA rate and fp32
    matrix-core rate (prune_probe_ceiling), with the shader clock measured
    during each, beside the datasheet peaks."""
    import ctypes as C
    from paper_1802_06625_amd import _lib as L

    def probe(kind, waves, size, reps):
        r = L.ProbeResult()
        L.call("prune_probe_ceiling", kind, waves, size, reps, C.byref(r))
        return r

    out = {}
    cp = {}
    for w in ((4, 8, 16) if sweep else (8,)):
        r = probe(L.PROBE_COPY, w, 1 << 30, 10)
        cp[w] = {"gbps": round(r.rate / 1e9, 1), "clock_ghz": round(r.clock_ghz, 3)}
    best = max(cp, key=lambda w: cp[w]["gbps"])
    out["copy"] = {"by_workgroups_per_cu": {str(k): v for k, v in cp.items()},
                   "gbps": cp[best]["gbps"], "bytes_per_launch": 2 * (1 << 30),
                   "clock_ghz": cp[best]["clock_ghz"], "datasheet_gbps": PEAK_HBM_GBPS,
                   "frac_of_datasheet": round(cp[best]["gbps"] / PEAK_HBM_GBPS, 4)}
    fma = {}
    for form, kind in (("chain", L.PROBE_FMA32), ("accumulate", L.PROBE_FMAC32),
                       ("chain_vgpr", L.PROBE_FMA3V), ("mixed", L.PROBE_FMAMIX)):
        for w in ((1, 2, 4, 8) if sweep else (2, 8)):
            r = probe(kind, w, 4096, 5)
            per_cu_cycle = r.rate / (r.n_cu * r.clock_ghz * 1e9) / 64.0 if r.clock_ghz else None
            fma[f"{form}_w{w}"] = {"tflops": round(2 * r.rate / 1e12, 2), "clock_ghz": round(r.clock_ghz, 3),
                                   "wave64_fma_per_cu_per_cycle": round(per_cu_cycle, 3) if per_cu_cycle else None}
    best = max(fma, key=lambda w: fma[w]["tflops"])
    out["fma32_unpacked"] = {"by_form_and_waves_per_simd": fma, "best": best,
                             "tflops": fma[best]["tflops"], "clock_ghz": fma[best]["clock_ghz"],
                             "wave64_fma_per_cu_per_cycle": fma[best]["wave64_fma_per_cu_per_cycle"],
                             "datasheet_tflops_packed": PEAK_FP32_VECTOR_TFLOPS,
                             "datasheet_tflops_unpacked": PEAK_FP32_VECTOR_TFLOPS / 2}
    mf = {}
    for w in ((1, 2, 4) if sweep else (2,)):
        r = probe(L.PROBE_MFMA32, w, 2048, 5)
        mf[w] = {"tflops": round(r.rate / 1e12, 2), "clock_ghz": round(r.clock_ghz, 3)}
    best = max(mf, key=lambda w: mf[w]["tflops"])
    out["mfma32"] = {"by_waves_per_simd": {str(k): v for k, v in mf.items()},
                     "tflops": mf[best]["tflops"], "clock_ghz": mf[best]["clock_ghz"],
                     "datasheet_tflops": PEAK_FP32_MATRIX_TFLOPS}
    return out


def algorithmic_flops(side, L):
    """Direct-form flops of the forward: per sample 4 (|x|) + K (8L + 3)."""
    n = side[:, 1].astype(np.float64)
    K = side[:, 0].astype(np.float64)
    return float(np.sum(n * (4.0 + K * (8.0 * L + 3.0))))


def cpu_baseline(wl, budget_s, gpu_first_frames):
    """The oracle as it stands, on the first frames of the same workload."""
    from oracle import graphs as og
    import synth

    cores = len(os.sched_getaffinity(0))
    # size the sample from a quick probe
    probe = 2
    sub = synth.Workload(wl.spec, wl.side[:, :probe].copy(),
                         wl.x[:, :int(wl.side[0, :probe, 1].sum())].copy(), wl.taps)
    t0 = time.perf_counter()
    og.run_plain(sub, C=3)
    dt = (time.perf_counter() - t0) / probe
    F_want = int(max(2, budget_s / max(dt, 1e-6)))
    if F_want <= wl.n_frames:
        F = F_want
        N = int(wl.side[0, :F, 1].sum())
        sub = synth.Workload(wl.spec, wl.side[:, :F].copy(), wl.x[:, :N].copy(), wl.taps)
        what = f"first {F} of {wl.n_frames} frames ({N} samples)"
    else:
        # the whole batch more than once, as one continuing stream: what
        # consecutive GPU steps fire
        reps = min(3, -(-F_want // wl.n_frames))
        F = reps * wl.n_frames
        sub = synth.Workload(wl.spec, np.concatenate([wl.side] * reps, axis=1),
                             np.concatenate([wl.x] * reps, axis=1), wl.taps)
        N = int(sub.side[0, :, 1].sum())
        what = (f"the whole batch of {wl.n_frames} frames {reps} times in a row as one continuing "
                f"stream, as consecutive steps fire it ({N} samples)")
    t0 = time.perf_counter()
    y, logs, _, _ = og.run_plain(sub, C=3)
    el = time.perf_counter() - t0
    # the GPU's first batch is kept for its first frames only
    Fc = min(F, gpu_first_frames.shape[0])
    Nc = int(wl.side[0, :Fc, 1].sum())
    gpu = gpu_first_frames[:Fc].reshape(-1)[:Nc].astype(np.complex128)
    rel = float(np.linalg.norm(gpu - y[:Nc]) / np.linalg.norm(y[:Nc]))
    return {"value": N / el / 1e6, "unit": "Msamples/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}, plain graph, C=3, float64 numpy, single thread ({cores} cores visible)",
            "seconds": round(el, 2), "gpu_rel_l2_on_first_frames": rel,
            "gpu_compared_frames": Fc}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs one graph on one GPU and this benchmark "
                                   "measures that single-GPU path; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd import ops
    from paper_1802_06625_amd.graph import PlainGraph

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.fb_variant:
        ops.set_variant(ops.variant_names().index(args.fb_variant) + 1)
    if args.only:
        fn = {"c1": lambda: bench_c1(args.steps, args.warmup),
              "perframe": lambda: bench_per_frame("C2"),
              "c3": lambda: bench_c3(args.steps, args.warmup),
              "c4": lambda: bench_direct("C4", args.steps, args.warmup),
              "c4fit": lambda: bench_fit(),
              "c5": lambda: bench_c5(args.steps, args.warmup),
              "c5bwd": lambda: bench_direct("C5", args.steps, args.warmup),
              "c2u": lambda: bench_c2_unfused(min(args.steps, 10), min(args.warmup, 5), None),
              "paper": lambda: bench_paper_dpd(min(args.steps, 10), min(args.warmup, 5)),
              "host": lambda: bench_host_stream(),
              "motion": lambda: bench_motion(min(args.steps, 10), min(args.warmup, 5))}[args.only]
        print(json.dumps({args.only: fn()}))
        return
    if args.ceilings:
        print(json.dumps({"ceilings": measure_ceilings(sweep=True)}))
        return
    if args.copy_calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b_ = torch.empty_like(a)
        for _ in range(2):
            b_.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read_per_dispatch": 1 << 30,
                          "copy_calib_bytes_written_per_dispatch": 1 << 30}))
        return
    print("bench: drawing C2 workload", file=sys.stderr, flush=True)
    wl = synth.make("C2", n_frames=args.frames or None)
    side = wl.side[0]
    F, n = side.shape[0], int(side[0, 1])
    Lt = wl.bank_L[0]
    samples = int(side[:, 1].sum())
    flops = algorithmic_flops(side, Lt)
    total_steps = 2 * (args.warmup + args.steps) + 16   # graph and stream-launch timings

    print("bench: building graph", file=sys.stderr, flush=True)
    pg = PlainGraph(wl.Kmax, wl.bank_L, n, F)
    g_variant = ops.autotuned_variant(Lt, wl.Kmax, n)
    g = pg.g
    analysis = analysis_summary(g)
    g.set_taps(pg.fb, torch.from_numpy(wl.taps[0]).cuda())
    pg.fifo_in.view(F, n).copy_(torch.from_numpy(wl.x[0]).view(F, n))
    del wl.x
    counts = side[:, 1]
    for _ in range(total_steps):
        g.source_push(pg.src, None, counts)
        g.config_push(pg.cfg, side)
    torch.cuda.synchronize()

    # first batch (kept for the oracle comparison), graph capture happens here
    g.fire(L.BATCHED_GRAPH, F)
    g.sync()
    first = pg.fifo_out.view(F, n)[: min(F, 1024)].cpu().numpy() if not args.profile_only else None
    print("bench: timing", file=sys.stderr, flush=True)

    # The batch as one hipGraph replay, and as the same launch sequence on the
    # stream, timed in alternating blocks; the step is reported in the faster
    # mode and both are listed.  During the stream-mode blocks the library
    # records HIP events around every forward-kernel launch on the launch
    # stream (the kernel's duration for the roofline; graph replays cannot be
    # timed from inside).
    ktime = [0.0, 0]

    def on_stream(on):
        if on:
            ops.timing_enable(True)
        else:
            ms_, n_ = ops.last_fb_kernel_ms()
            ktime[0] += ms_
            ktime[1] += n_
            ops.timing_enable(False)

    graph_ev, stream_ev, graph_ms, stream_ms = _time_modes(
        lambda: g.fire(L.BATCHED_GRAPH, F), lambda: g.fire(L.BATCHED, F), args.steps, args.warmup,
        on_stream, with_wall=True)
    g.sync()
    k_total_ms, k_launches = ktime
    if graph_ms <= stream_ms:
        mode_name, ms_step, ev_ms_step = "batched_graph", graph_ms, graph_ev
    else:
        mode_name, ms_step, ev_ms_step = "batched_stream", stream_ms, stream_ev
    value = samples / (ms_step * 1e-3) / 1e6

    out = {"metric": METRIC, "value": round(value, 1), "unit": "Msamples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"plain single-stream graph src->config->filterbank->sink, "
                                  f"{F} frames x {n} complex64 samples, K~U{{1..10}} per frame "
                                  f"from control tokens, L={Lt} taps, one batched firing per step",
                      "frames": F, "frame_len": n, "taps": Lt, "Kmax": wl.Kmax,
                      "samples_per_step": samples, "mode": mode_name,
                      "fb_variant": ops.variant_names()[g_variant - 1] if g_variant else None},
           "event_ms_per_step": round(ev_ms_step, 4),
           "batched_graph_msamples": round(samples / (graph_ms * 1e-3) / 1e6, 1),
           "batched_stream_msamples": round(samples / (stream_ms * 1e-3) / 1e6, 1),
           "analysis": analysis}
    if args.profile_only:
        print(json.dumps(out))
        return

    # forward-kernel duration: the average over the stream-mode timed steps
    k_ms = k_total_ms / max(k_launches, 1)
    achieved = flops / (k_ms * 1e-3) / 1e12
    traffic = measured_traffic(os.path.join(ROOT, "paper_1802_06625_amd", "csrc", "fb_forward.hip"),
                               os.path.join(ROOT, "profiles", "fb_forward_c2_traffic.txt"))
    # what the Horner kernel executes: 2(KH-1)+4 fp32 FMAs per output and tap
    # (KH = highest active branch, K under prefix masks), beside the measured
    # ceiling of all-register fp32 FMAs (two-operand accumulate form, 8 waves
    # per SIMD) on this device
    from paper_1802_06625_amd import _lib as Lb
    import ctypes as C
    fma_lanes = float(np.sum(side[:, 1].astype(np.float64) * Lt * (2.0 * side[:, 0] + 2.0)))
    pr = Lb.ProbeResult()
    Lb.call("prune_probe_ceiling", Lb.PROBE_FMAC32, 8, 4096, 5, C.byref(pr))
    ceil_tf = 2.0 * pr.rate / 1e12
    exec_tf = 2.0 * fma_lanes / (k_ms * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "achieved": round(achieved, 2),
                       "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": traffic,
                       "traffic_algorithmic": 16.0 * samples,
                       "kernel": "k_fb_forward", "kernel_ms": round(k_ms, 4),
                       "kernel_launches_timed": k_launches,
                       "algorithmic_flops_per_launch": flops,
                       "hbm_gbps_algorithmic": round(16.0 * samples / (k_ms * 1e-3) / 1e9, 1),
                       "executed": {"fma_lanes_per_launch": fma_lanes, "tflops": round(exec_tf, 2),
                                    "measured_fp32_fma_ceiling_tflops": round(ceil_tf, 2),
                                    "ceiling_clock_ghz": round(pr.clock_ghz, 3),
                                    "frac_of_measured_ceiling": round(exec_tf / ceil_tf, 4)}}

    del g, pg
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_per_frame:
        print("bench: per-frame firing", file=sys.stderr, flush=True)
        pf = bench_per_frame("C2")
        out["per_frame"] = pf
        out["per_frame_msamples"] = pf["msamples_mean"]
        out["batched_vs_per_frame"] = round(value / pf["msamples_mean"], 1)
    if not args.only_c2:
        print("bench: plain graph, 64 frames", file=sys.stderr, flush=True)
        out["c1"] = bench_c1(args.steps, args.warmup)
        print("bench: unfused DPD graph", file=sys.stderr, flush=True)
        out["c2_unfused"] = bench_c2_unfused(min(args.steps, 10), min(args.warmup, 5), ms_step)
        print("bench: motion detection", file=sys.stderr, flush=True)
        out["motion_1080p"] = bench_motion(min(args.steps, 10), min(args.warmup, 5))
        print("bench: host source and sink over PCIe", file=sys.stderr, flush=True)
        out["c2_host_stream"] = bench_host_stream()
        print("bench: the paper's DPD shape", file=sys.stderr, flush=True)
        out["paper_dpd"] = bench_paper_dpd(min(args.steps, 10), min(args.warmup, 5))
        print("bench: fwd+bwd (differentiation workload)", file=sys.stderr, flush=True)
        out["c4_fwd_bwd"] = bench_direct("C4", args.steps, args.warmup)
        out["c4_fit"] = bench_fit()
        print("bench: batched uneven frames", file=sys.stderr, flush=True)
        out["c3_batched"] = bench_c3(args.steps, args.warmup)
        print("bench: routed multi-stream graph", file=sys.stderr, flush=True)
        out["c5_routed"] = bench_c5(args.steps, args.warmup)
        out["c5_fwd_bwd"] = bench_direct("C5", args.steps, args.warmup)

    if not args.no_cpu_baseline:
        print("bench: oracle baseline", file=sys.stderr, flush=True)
        wl2 = synth.make("C2", n_frames=args.frames or None)
        out["cpu_baseline"] = cpu_baseline(wl2, args.cpu_seconds, first)
        if not args.only_c2:
            out["oracle_timings"] = oracle_timings()
    print(json.dumps(out))


def bench_per_frame(name, C=3, warm=3, runs=8, frames=None):
    """The paper's execution model as the baseline: one decode and one
    filter-bank launch per firing, in host order, through FIFOs of C = 3
    blocks (the paper's triple buffering), frames resident in HBM.  A run
    fires the whole batch; 3 warm-up runs, then 8 timed runs (host clock
    around each, device synchronised on both sides), mean and median."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd.graph import PlainGraph
    wl = synth.make(name, n_frames=frames)
    side = wl.side[0]
    n = side[:, 1].astype(np.int64)
    F = len(n)
    param = bool(np.any(n != n[0]))
    atr = int(wl.spec.n_max) if param else int(n[0])
    pg = PlainGraph(wl.Kmax, wl.bank_L, atr, C, param)
    g = pg.g
    g.set_taps(pg.fb, torch.from_numpy(wl.taps[0]).cuda())
    x = torch.from_numpy(wl.x[0]).cuda()
    samples = int(n.sum())
    times = []
    for r in range(warm + runs):
        g.source_push(pg.src, x, n)
        g.config_push(pg.cfg, side)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.fire(L.PER_FIRING)
        torch.cuda.synchronize()
        if r >= warm:
            times.append(time.perf_counter() - t0)
        g.sync()
    rates = [samples / t / 1e6 for t in times]
    res = {"workload": f"{wl.spec.description}; per-frame firing, C={C}", "frames": F,
           "samples": samples, "runs": runs, "warmup_runs": warm,
           "msamples_mean": round(float(np.mean(rates)), 2),
           "msamples_median": round(float(np.median(rates)), 2),
           "seconds_per_run_mean": round(float(np.mean(times)), 4)}
    del g, pg, x
    torch.cuda.empty_cache()
    return res


def bench_c1(steps, warmup):
    """The small plain graph (64 frames x 1024, K~U{1..4}, L=8): absolute
    numbers, batched (both launch modes) and per-frame with C = 3."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd.graph import PlainGraph
    wl = synth.make("C1")
    side = wl.side[0]
    F, n = side.shape[0], int(side[0, 1])
    pg = PlainGraph(wl.Kmax, wl.bank_L, n, F)
    g = pg.g
    g.set_taps(pg.fb, torch.from_numpy(wl.taps[0]).cuda())
    pg.fifo_in.view(F, n).copy_(torch.from_numpy(wl.x[0]).view(F, n))
    for _ in range(2 * (steps + warmup) + 1):
        g.source_push(pg.src, None, side[:, 1])
        g.config_push(pg.cfg, side)
    torch.cuda.synchronize()
    g.fire(L.BATCHED_GRAPH, F)
    ms_graph, ms_stream = _time_modes(lambda: g.fire(L.BATCHED_GRAPH, F), lambda: g.fire(L.BATCHED, F),
                                      steps, warmup)
    g.sync()
    ms = min(ms_graph, ms_stream)
    samples = F * n
    res = {"workload": wl.spec.description, "samples": samples,
           "msamples": round(samples / (ms * 1e-3) / 1e6, 1), "ms_per_batch": round(ms, 4),
           "mode": "batched_graph" if ms_graph <= ms_stream else "batched_stream",
           "graph_ms": round(ms_graph, 4), "stream_ms": round(ms_stream, 4)}
    del g, pg
    torch.cuda.empty_cache()
    res["per_frame"] = bench_per_frame("C1")
    res["batched_vs_per_frame"] = round(res["msamples"] / res["per_frame"]["msamples_mean"], 1)
    return res


def _time_events(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _time_modes(fire_graph, fire_stream, steps, warmup, on_stream=None, with_wall=False):
    """Milliseconds per step of the two batched launch modes: both warmed up
    first, then timed in blocks ordered graph, stream, stream, graph, so that
    neither mode lands in the other's warm-up and a clock that still drifts
    during the timed region weighs on both modes alike.  on_stream(True/False)
    brackets every stream-mode block (kernel timing).  with_wall: also the
    host wall-clock milliseconds per step of each mode, each block bracketed
    by device synchronisations."""
    import torch
    for _ in range(warmup):
        fire_graph()
        fire_stream()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    nb = 2 if steps >= 2 else 1
    sizes = [steps // nb + (1 if b < steps % nb else 0) for b in range(nb)]
    tot = {"graph": 0.0, "stream": 0.0}
    wall = {"graph": 0.0, "stream": 0.0}
    for b, k in enumerate(sizes):
        order = (("graph", fire_graph), ("stream", fire_stream))
        for name, fn in (order if b % 2 == 0 else order[::-1]):
            if name == "stream" and on_stream:
                on_stream(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(st)
            for _ in range(k):
                fn()
            e1.record(st)
            torch.cuda.synchronize()
            wall[name] += time.perf_counter() - t0
            tot[name] += e0.elapsed_time(e1)
            if name == "stream" and on_stream:
                on_stream(False)
    if with_wall:
        return (tot["graph"] / steps, tot["stream"] / steps,
                wall["graph"] * 1e3 / steps, wall["stream"] * 1e3 / steps)
    return tot["graph"] / steps, tot["stream"] / steps


def bench_fit(steps=200, lr=1e-2):
    """The differentiation workload as a tap fit: full-batch Adam on the taps
    of the amplifier-fit workload (256 x 8192, K=8, L=16) through the
    autograd Function (forward + grad_taps kernels), loss computed in torch.
    The step time includes torch's loss and Adam kernels; the target's noise
    (per-component sigma 0.01) puts the loss floor near 2e-4."""
    import torch
    import synth
    from paper_1802_06625_amd import ops
    wl = synth.make("C4")
    rows = ops.frames_from_side(wl.side, wl.Kmax, False)
    fr = ops.frame_table(rows)
    mfl = int(wl.side[:, :, 1].max())
    x = torch.from_numpy(wl.x).cuda()
    target = torch.from_numpy(wl.target).cuda()
    taps = torch.nn.Parameter(torch.from_numpy(wl.taps).cuda().clone())
    opt = torch.optim.Adam([taps], lr=lr)

    def step():
        y = ops.filter_bank(x, taps, fr, wl.Kmax, wl.bank_L, mfl)
        e = y - target
        loss = torch.mean(e.real ** 2 + e.imag ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        return loss

    losses = [float(step().detach())]     # first step untimed (allocations)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st = torch.cuda.current_stream()
    vals = []
    e0.record(st)
    for _ in range(steps - 1):
        vals.append(step().detach())
    e1.record(st)
    torch.cuda.synchronize()
    losses += [float(v) for v in vals]
    ms = e0.elapsed_time(e1) / (steps - 1)
    samples = int(wl.x.size)
    return {"workload": wl.spec.description + f", {steps} Adam steps lr {lr}",
            "ms_per_step": round(ms, 4), "msamples_per_s": round(samples / (ms * 1e-3) / 1e6, 1),
            "loss_by_step": {str(k): round(losses[k], 6) for k in (0, 10, 50, 100, steps - 1)},
            "loss_noise_floor": 2e-4}


def bench_direct(name, steps, warmup):
    """Forward and forward+adjoint of the filter bank over whole streams
    (prune_fb_forward / prune_fb_backward) on a workload; the cotangent is the
    workload's seeded one."""
    import torch
    import synth
    from paper_1802_06625_amd import ops
    wl = synth.make(name, cotangent=True)
    S, N = wl.x.shape
    routed = wl.spec.pass_prob > 0
    rows = ops.frames_from_side(wl.side, wl.Kmax, routed)
    fr = ops.frame_table(rows)
    mfl = int(wl.side[:, :, 1].max())
    x = torch.from_numpy(wl.x).cuda()
    taps = torch.from_numpy(wl.taps).cuda()
    gy = torch.from_numpy(wl.gy).cuda()
    y, gx, gt = torch.empty_like(x), torch.empty_like(x), torch.empty_like(taps)
    work = torch.empty(ops.workspace_bytes(S, N, wl.Kmax, wl.bank_L, len(rows), mfl), dtype=torch.uint8,
                       device="cuda")
    fwd = lambda: ops.fb_forward(x, taps, fr, wl.Kmax, wl.bank_L, mfl, y=y)
    bwd = lambda: ops.fb_backward(x, taps, fr, gy, wl.Kmax, wl.bank_L, mfl, gx=gx, gt=gt, work=work)
    # the adjoint as a tap fit uses it: grad_taps only (grad_x not computed)
    bwd_taps = lambda: ops.fb_backward(x, taps, fr, gy, wl.Kmax, wl.bank_L, mfl, gt=gt, work=work,
                                       want_gx=False)
    t_f = _time_events(fwd, steps, warmup)
    t_b = _time_events(bwd, steps, warmup)
    t_bt = _time_events(bwd_taps, steps, warmup)
    bwd_by_form = {}
    for form in (1, 2, 3):
        ops.set_bwd_variant(form)
        try:
            bwd_by_form[ops.bwd_variant_name(form)] = round(_time_events(bwd, steps, warmup), 4)
        finally:
            ops.set_bwd_variant(0)
    by_variant = {}
    if name in ("C4", "C5"):
        # every forward kernel forced in turn (vector Horner and matrix-core
        # block-Toeplitz), same launch configuration as the autotuned call
        for v, vname in enumerate(ops.variant_names(), start=1):
            ops.set_variant(v)
            try:
                by_variant[vname] = round(_time_events(fwd, steps, warmup), 4)
            finally:
                ops.set_variant(0)
    L = wl.bank_L[0]
    side = wl.side.reshape(-1, 4)
    fb_n = np.array([n for (_, _, n, _, r) in rows if not r], dtype=np.float64)
    fb_k = np.array([wl.Kmax if routed else int(side[k, 0]) for k, (_, _, n, _, r) in enumerate(rows) if not r],
                    dtype=np.float64)
    f_fwd = float(np.sum(fb_n * (4.0 + fb_k * (8.0 * L + 3.0))))
    f_bwd = float(np.sum(fb_n * (10.0 + fb_k * (16.0 * L + 17.0))))
    samples = S * N
    res = {"workload": wl.spec.description, "samples": samples,
           "fwd_msamples": round(samples / (t_f * 1e-3) / 1e6, 1),
           "fwd_bwd_msamples": round(samples / ((t_f + t_b) * 1e-3) / 1e6, 1),
           "fwd_ms": round(t_f, 4), "bwd_ms": round(t_b, 4),
           "fwd_bwd_taps_only_msamples": round(samples / ((t_f + t_bt) * 1e-3) / 1e6, 1),
           "bwd_taps_only_ms": round(t_bt, 4),
           "fwd_tflops_alg": round(f_fwd / (t_f * 1e-3) / 1e12, 2),
           "bwd_tflops_alg": round(f_bwd / (t_b * 1e-3) / 1e12, 2),
           "fwd_bwd_frac_of_fp32_vector_peak": round((f_fwd + f_bwd) / ((t_f + t_b) * 1e-3) / 1e12
                                                      / PEAK_FP32_VECTOR_TFLOPS, 4),
           "fwd_variant": ops.variant_names()[ops.tuned_variant(x, fr, wl.Kmax, wl.bank_L, mfl) - 1],
           "bwd_form": ops.bwd_variant_name(ops.autotuned_bwd_variant(L, wl.Kmax, mfl)),
           "bwd_ms_by_form": bwd_by_form}
    if by_variant:
        res["fwd_ms_by_variant"] = by_variant
        res["fwd_tflops_alg_by_variant"] = {k: round(f_fwd / (v * 1e-3) / 1e12, 2)
                                            for k, v in by_variant.items()}
    # accuracy of what was timed: one more forward and adjoint in the timed
    # configuration, against the oracle on the compared streams
    fwd()
    bwd()
    torch.cuda.synchronize()
    res["accuracy"] = direct_accuracy(wl, y, gx, gt, streams=range(min(S, 4)))
    if name == "C5":
        # matrix-core kernel (block-Toeplitz form): the fastest of its
        # variants, kernel duration from the library's HIP events on the
        # launch stream
        names = ops.variant_names()
        mv = min((k for k in by_variant if k.startswith("mfma")), key=by_variant.get)
        ops.set_variant(names.index(mv) + 1)
        try:
            for _ in range(warmup):
                fwd()
            torch.cuda.synchronize()
            ops.timing_enable(True)
            for _ in range(steps):
                fwd()
            torch.cuda.synchronize()
            tot, nl = ops.last_fb_kernel_ms()
        finally:
            ops.timing_enable(False)
            ops.set_variant(0)
        k_ms = tot / max(nl, 1)
        ach = f_fwd / (k_ms * 1e-3) / 1e12
        res["roofline_mfma"] = {"bound": "mfma", "kernel": "k_fb_mfma", "variant": mv,
                                "achieved": round(ach, 2), "peak": PEAK_FP32_MATRIX_TFLOPS,
                                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_MATRIX_TFLOPS, 4),
                                "kernel_ms": round(k_ms, 4), "algorithmic_flops_per_launch": f_fwd}
    del x, taps, gy, y, gx, gt, work
    torch.cuda.empty_cache()
    return res


def direct_accuracy(wl, y, gx, gt, streams):
    """Relative L2 error (Re and Im as reals) of the device forward output,
    input gradient and tap gradient against the FP64 oracle's closed forms,
    over the given streams (each in full)."""
    from oracle.filterbank import fb_stream, fb_stream_adjoint
    from oracle.graphs import stream_frames
    yd, gxd, gtd = y.cpu().numpy(), gx.cpu().numpy(), gt.cpu().numpy()
    err = {"y": [0.0, 0.0], "grad_x": [0.0, 0.0], "grad_taps": [0.0, 0.0]}
    streams = list(streams)
    for s_ in streams:
        fr = stream_frames(wl, s_)
        ry = fb_stream(wl.x[s_], fr, wl.taps[s_], wl.bank_L, wl.Kmax)
        rx, rt = fb_stream_adjoint(wl.x[s_], fr, wl.taps[s_], wl.bank_L, wl.Kmax, wl.gy[s_])
        for k, a, b in (("y", yd[s_], ry), ("grad_x", gxd[s_], rx), ("grad_taps", gtd[s_], rt)):
            d = np.asarray(a, np.complex128) - b
            err[k][0] += float(np.vdot(d, d).real)
            err[k][1] += float(np.vdot(b, b).real)
    out = {k: float(np.sqrt(v[0] / v[1])) for k, v in err.items()}
    out["streams_compared"] = len(streams)
    out["samples_compared"] = int(len(streams) * wl.x.shape[1])
    return out


def oracle_timings():
    """The oracle as it stands (numpy FP64, single thread) on the other
    workloads: the 64-frame plain graph and the differentiation workload in
    full, the uneven-frame and wide multi-stream workloads on their first 64
    frames.  Msamples/s of input."""
    import synth
    from oracle import graphs as og
    from oracle.filterbank import fb_stream, fb_stream_adjoint
    from oracle.graphs import stream_frames
    cores = len(os.sched_getaffinity(0))
    res = {"cores": 1, "cores_visible": cores, "kind": "oracle", "precision": "float64"}
    wl = synth.make("C1")
    t0 = time.perf_counter()
    og.run_plain(wl, C=3)
    el = time.perf_counter() - t0
    res["c1_graph_full"] = {"samples": int(wl.x.size), "seconds": round(el, 4),
                            "msamples": round(wl.x.size / el / 1e6, 3)}
    wl = synth.make("C4", cotangent=True)
    fr = stream_frames(wl, 0)
    t0 = time.perf_counter()
    fb_stream(wl.x[0], fr, wl.taps[0], wl.bank_L, wl.Kmax)
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    fb_stream_adjoint(wl.x[0], fr, wl.taps[0], wl.bank_L, wl.Kmax, wl.gy[0])
    tb = time.perf_counter() - t0
    res["c4_full"] = {"samples": int(wl.x.size), "fwd_seconds": round(tf, 3), "bwd_seconds": round(tb, 3),
                      "fwd_msamples": round(wl.x.size / tf / 1e6, 3),
                      "fwd_bwd_msamples": round(wl.x.size / (tf + tb) / 1e6, 3)}
    wl = synth.make("C3")
    n64 = int(wl.side[0, :64, 1].sum())
    sub = synth.Workload(wl.spec, wl.side[:, :64].copy(), wl.x[:, :n64].copy(), wl.taps)
    t0 = time.perf_counter()
    og.run_plain(sub, C=3)
    el = time.perf_counter() - t0
    res["c3_first_64_frames"] = {"samples": n64, "seconds": round(el, 3), "msamples": round(n64 / el / 1e6, 3)}
    wl = synth.make("C5", cotangent=True)
    S64 = 64 // wl.n_frames
    t0 = time.perf_counter()
    for s_ in range(S64):
        fb_stream(wl.x[s_], stream_frames(wl, s_), wl.taps[s_], wl.bank_L, wl.Kmax)
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    for s_ in range(S64):
        fb_stream_adjoint(wl.x[s_], stream_frames(wl, s_), wl.taps[s_], wl.bank_L, wl.Kmax, wl.gy[s_])
    tb = time.perf_counter() - t0
    n = S64 * wl.x.shape[1]
    res["c5_first_64_frames"] = {"samples": n, "streams": S64, "fwd_seconds": round(tf, 3),
                                 "bwd_seconds": round(tb, 3), "fwd_msamples": round(n / tf / 1e6, 3),
                                 "fwd_bwd_msamples": round(n / (tf + tb) / 1e6, 3)}
    return res


def analysis_summary(g):
    """Compile-time analysis of a workload graph (prune_graph_analyze, host
    code): its size, what it found and how long it took."""
    t0 = time.perf_counter()
    rep = g.analyze()
    ms = (time.perf_counter() - t0) * 1e3
    return {"actors": len(rep["dc_of_actor"]), "fifos": len(rep["beta"]), "dpgs": len(rep["dpgs"]),
            "dcs": len(rep["dcs"]), "violations": len(rep["violations"]), "ms": round(ms, 3)}


def bench_c2_unfused(steps, warmup, fused_ms):
    """The headline batch through the DPD graph before actor merging
    (poly -> 10 FIR actors -> add, per-branch device FIFOs): what merging
    the dynamic processing graph into one actor buys."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd.graph import UnfusedGraph
    wl = synth.make("C2")
    side = wl.side[0]
    F, n = side.shape[0], int(side[0, 1])
    ug = UnfusedGraph(wl.Kmax, wl.bank_L[0], n, F)
    g = ug.g
    ug.set_taps(torch.from_numpy(wl.taps[0, 0]).cuda())
    ug.fifo_in.view(F, n).copy_(torch.from_numpy(wl.x[0]).view(F, n))
    del wl.x
    for _ in range(2 * (steps + warmup) + 1):
        g.source_push(ug.src, None, side[:, 1])
        g.config_push(ug.cfg, side)
    torch.cuda.synchronize()
    g.fire(L.BATCHED_GRAPH, F)
    ms_graph, ms_stream = _time_modes(lambda: g.fire(L.BATCHED_GRAPH, F), lambda: g.fire(L.BATCHED, F),
                                      steps, warmup)
    g.sync()
    ms = min(ms_graph, ms_stream)
    samples = F * n
    fifo_bytes = sum(g.required_bytes(f) for f in [ug.f_in, ug.f_out] + ug.f_win + ug.f_br)
    res = {"workload": "the headline batch (4096 x 16384, K~U{1..10}, L=32) through the unfused "
                       "DPD graph: poly -> 10 FIR_b -> add with per-branch device FIFOs",
           "msamples": round(samples / (ms * 1e-3) / 1e6, 1), "ms_per_batch": round(ms, 4),
           "mode": "batched_graph" if ms_graph <= ms_stream else "batched_stream",
           "graph_ms": round(ms_graph, 4), "stream_ms": round(ms_stream, 4),
           "fifo_gib": round(fifo_bytes / 2**30, 2),
           "merged_speedup": round(ms / fused_ms, 2) if fused_ms else None}
    del g, ug
    torch.cuda.empty_cache()
    return res


# The paper's DPD throughput with PRUNE on its heterogeneous platforms
# (complex-float Msamples/s, Table IV): context for the same graph shape.
PAPER_DPD_MSAMPLES = {"AMD Radeon RX 460 (PCIe)": 106.0, "AMD Carrizo R7 iGPU": 39.5,
                      "Intel i7-6700HQ OpenCL": 25.1}


def bench_paper_dpd(steps, warmup):
    """The shape of the paper's DPD run (1024 frames x 65536, K~U{2..10},
    L=10, 2^26 samples) through the merged filter bank and through the
    unfused graph of the paper (poly -> 10 FIR_b -> add)."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd.graph import PlainGraph, UnfusedGraph
    wl = synth.make("P")
    side = wl.side[0]
    F, n = side.shape[0], int(side[0, 1])
    x = torch.from_numpy(wl.x[0]).cuda()
    taps = torch.from_numpy(wl.taps[0]).cuda()
    del wl.x
    res = {"workload": wl.spec.description, "samples": F * n}
    for name in ("merged", "unfused"):
        if name == "merged":
            G = PlainGraph(wl.Kmax, wl.bank_L, n, F)
            G.g.set_taps(G.fb, taps)
        else:
            G = UnfusedGraph(wl.Kmax, wl.bank_L[0], n, F)
            G.set_taps(taps[0])
        g = G.g
        G.fifo_in.view(F, n).copy_(x.view(F, n))
        for _ in range(2 * (steps + warmup) + 1):
            g.source_push(G.src, None, side[:, 1])
            g.config_push(G.cfg, side)
        torch.cuda.synchronize()
        g.fire(L.BATCHED_GRAPH, F)
        ms_graph, ms_stream = _time_modes(lambda: g.fire(L.BATCHED_GRAPH, F),
                                          lambda: g.fire(L.BATCHED, F), steps, warmup)
        g.sync()
        ms = min(ms_graph, ms_stream)
        res[name] = {"msamples": round(F * n / (ms * 1e-3) / 1e6, 1), "ms_per_batch": round(ms, 4),
                     "mode": "batched_graph" if ms_graph <= ms_stream else "batched_stream"}
        del g, G
        torch.cuda.empty_cache()
    res["paper_prune_heterogeneous_msamples"] = PAPER_DPD_MSAMPLES
    return res


def bench_host_stream(batch=512):
    """The headline workload with a host source and sink
    (prune_graph_stream_host): frames from pinned host memory, outputs back
    to pinned host memory, copies in both directions overlapped with the
    firing.  PCIe-inclusive; the headline value keeps inputs in HBM."""
    import torch
    import synth
    from paper_1802_06625_amd.graph import PlainGraph
    wl = synth.make("C2")
    side = wl.side[0]
    F, n = side.shape[0], int(side[0, 1])
    hin = torch.from_numpy(wl.x[0]).pin_memory()
    del wl.x
    hout = torch.empty(hin.shape, dtype=hin.dtype).pin_memory()
    pg = PlainGraph(wl.Kmax, wl.bank_L, n, 2 * batch)
    g = pg.g
    g.set_taps(pg.fb, torch.from_numpy(wl.taps[0]).cuda())
    # one warm pass over the first batches, then the timed pass over all frames
    g.stream_host(pg.src, pg.cfg, pg.snk, hin[:4 * batch * n], side[:4 * batch], hout[:4 * batch * n], batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.stream_host(pg.src, pg.cfg, pg.snk, hin, side, hout, batch)
    sec = time.perf_counter() - t0
    samples = F * n
    res = {"workload": "the headline batch streamed from and to pinned host memory in batches of "
                       f"{batch} frames (FIFOs hold two batches)",
           "msamples_pcie_inclusive": round(samples / sec / 1e6, 1), "seconds": round(sec, 4),
           "host_bytes_each_way": samples * 8,
           "gb_per_s_each_way": round(samples * 8 / sec / 1e9, 2)}
    del g, pg
    torch.cuda.empty_cache()
    return res


# The paper's Motion Detection throughput with PRUNE on its heterogeneous
# platforms (1080p frames/s, Table III): context for the same graph.
PAPER_MOTION_FPS = {"AMD Radeon RX 460 (PCIe)": 772.0, "AMD Carrizo R7 iGPU": 140.0,
                    "Intel i7-6700HQ OpenCL": 113.0}


def bench_motion(steps, warmup, batch=64):
    """Motion Detection (Gauss 5x5 -> Thres with a one-frame delay -> Med 5)
    on synthetic 8-bit 1920x1080 frames, batched, frames resident in HBM."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd.graph import MotionGraph
    W, H = 1920, 1080
    v = synth.make_video(8)
    mg = MotionGraph(W, H, batch + 1)
    g = mg.g
    npix = W * H
    blocks = mg.fifo_in.view(-1, npix)
    for f in range(batch):
        blocks[f].copy_(torch.from_numpy(v[f % len(v)].reshape(-1)))
    for _ in range(2 * (steps + warmup) + 1):
        g.source_push(mg.src, None, np.full(batch, npix))
    torch.cuda.synchronize()
    g.fire(L.BATCHED_GRAPH, batch)
    ms_graph, ms_stream = _time_modes(lambda: g.fire(L.BATCHED_GRAPH, batch),
                                      lambda: g.fire(L.BATCHED, batch), steps, warmup)
    g.sync()
    ms = min(ms_graph, ms_stream)
    fps = batch / (ms * 1e-3)
    # HBM bytes per frame: source block read by Gauss, Gauss output written to
    # two FIFOs, both read by Thres, Thres output written and read by Med,
    # Med output written
    bytes_per_frame = 7 * npix
    res = {"workload": f"1920x1080 8-bit frames, batches of {batch}, Gauss 5x5 -> Thres (one-frame "
                       "delay FIFO) -> Med 5", "frames_per_s": round(fps, 1),
           "ms_per_batch": round(ms, 4), "mode": "batched_graph" if ms_graph <= ms_stream else "batched_stream",
           "hbm_gbps_algorithmic": round(bytes_per_frame * fps / 1e9, 1),
           "hbm_frac_of_8tbs": round(bytes_per_frame * fps / 8e12, 3),
           "paper_prune_heterogeneous_fps": PAPER_MOTION_FPS}
    del g, mg
    torch.cuda.empty_cache()
    return res


def bench_c3(steps, warmup):
    """Batched uneven frames: 2048 frames with log-uniform rates in
    [256, 65536], three tap banks, one hipGraph replay per batch."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd.graph import PlainGraph
    wl = synth.make("C3")
    side = wl.side[0]
    F, atr = side.shape[0], int(wl.spec.n_max)
    n = side[:, 1].astype(np.int64)
    pg = PlainGraph(wl.Kmax, wl.bank_L, atr, F, param=True)
    g = pg.g
    g.set_taps(pg.fb, torch.from_numpy(wl.taps[0]).cuda())
    off = np.concatenate([[0], np.cumsum(n)])
    x = torch.from_numpy(wl.x[0]).cuda()
    blocks = pg.fifo_in.view(F, atr)
    for f in range(F):
        blocks[f, :n[f]] = x[off[f]:off[f + 1]]
    del x
    for _ in range(2 * (steps + warmup) + 1):
        g.source_push(pg.src, None, n)
        g.config_push(pg.cfg, side)
    torch.cuda.synchronize()
    g.fire(L.BATCHED_GRAPH, F)
    ms_graph, ms_stream = _time_modes(lambda: g.fire(L.BATCHED_GRAPH, F), lambda: g.fire(L.BATCHED, F),
                                      steps, warmup)
    g.sync()
    ms = min(ms_graph, ms_stream)
    samples = int(n.sum())
    # accuracy of the last timed batch on its first 64 frames: the oracle on
    # those frames with the previous batch's last samples as the history
    from oracle.filterbank import fb_stream
    from oracle.graphs import stream_frames
    H = max(wl.bank_L) - 1
    fr64 = stream_frames(wl, 0)[:64]
    n64 = int(sum(f[1] for f in fr64))
    xc = np.concatenate([wl.x[0, samples - H:samples], wl.x[0, :n64]])
    ref = fb_stream(xc, [(0, H, 0, 0)] + [(t0 + H, m, k, r) for (t0, m, k, r) in fr64], wl.taps[0],
                    wl.bank_L, wl.Kmax)[H:]
    dev = np.concatenate([pg.fifo_out.view(F, atr)[f, :n[f]].cpu().numpy() for f in range(64)])
    rel64 = float(np.linalg.norm(dev.astype(np.complex128) - ref) / np.linalg.norm(ref))
    Lb = np.array(wl.bank_L, dtype=np.float64)[side[:, 2]]
    flops = float(np.sum(n * (4.0 + side[:, 0] * (8.0 * Lb + 3.0))))
    res = {"workload": wl.spec.description, "samples": samples, "frames": F,
           "msamples": round(samples / (ms * 1e-3) / 1e6, 1), "ms_per_batch": round(ms, 4),
           "mode": "batched_graph" if ms_graph <= ms_stream else "batched_stream",
           "graph_ms": round(ms_graph, 4), "stream_ms": round(ms_stream, 4),
           "tflops_alg": round(flops / (ms * 1e-3) / 1e12, 2),
           "frac_of_fp32_vector_peak": round(flops / (ms * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4),
           "rel_l2_first_64_frames_of_last_batch": rel64}
    del g, pg
    torch.cuda.empty_cache()
    return res


def bench_c5(steps, warmup):
    """Routed multi-stream graph: 64 independent switch/filter-bank/
    passthrough/select streams of 16 frames x 32768, one hipGraph replay for
    all streams."""
    import torch
    import synth
    from paper_1802_06625_amd import _lib as L
    from paper_1802_06625_amd import ops
    from paper_1802_06625_amd.graph import RoutedGraph
    wl = synth.make("C5")
    S, F, n = wl.n_streams, wl.n_frames, int(wl.side[0, 0, 1])
    rg = RoutedGraph(S, wl.Kmax, wl.bank_L, n, F)
    g = rg.g
    analysis = analysis_summary(g)
    for s, ids in enumerate(rg.streams):
        g.set_taps(ids["fb"], torch.from_numpy(wl.taps[s]).cuda())
        rg.storage[s]["in"].view(F, n).copy_(torch.from_numpy(wl.x[s]).view(F, n))
        for _ in range(2 * (steps + warmup) + 1):
            g.source_push(ids["src"], None, wl.side[s, :, 1])
            g.config_push(ids["cfg"], wl.side[s])
    torch.cuda.synchronize()
    g.fire(L.BATCHED_GRAPH, F)
    ms_graph, ms_stream = _time_modes(lambda: g.fire(L.BATCHED_GRAPH, F), lambda: g.fire(L.BATCHED, F),
                                      steps, warmup)
    g.sync()
    ms = min(ms_graph, ms_stream)
    samples = S * F * n
    n_fb = int((wl.side[:, :, 3] == 0).sum())
    Lt = wl.bank_L[0]
    flops = float(n_fb * n * (4.0 + wl.Kmax * (8.0 * Lt + 3.0)))
    res = {"workload": wl.spec.description, "samples": samples,
           "passthrough_frames": int(S * F - n_fb),
           "msamples": round(samples / (ms * 1e-3) / 1e6, 1), "ms_per_batch": round(ms, 4),
           "mode": "batched_graph" if ms_graph <= ms_stream else "batched_stream",
           "graph_ms": round(ms_graph, 4), "stream_ms": round(ms_stream, 4),
           "tflops_alg": round(flops / (ms * 1e-3) / 1e12, 2),
           "fb_variant": ops.variant_names()[ops.autotuned_variant(Lt, wl.Kmax, n) - 1],
           "analysis": analysis}
    del g, rg
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
