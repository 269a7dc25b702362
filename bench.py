#!/usr/bin/env python3
"""Throughput of the batched VELO GNN track-finding path on one MI355X.

One step = one call of the whole path (embedding, rough graph, GNN, edge cut,
components) over one batch of synthetic events already resident in HBM.
Prints ONE JSON line with events/s at the headline precision, the same
workload at the other precisions, the roofline of the dominant kernel
(measured with HIP events on the library's stream over the timed region),
the float64 CPU oracle timed on a bounded sample of the same workload, and
the plain per-event float32 path (one call per event).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch256]
                       [--precision fp32|bf16] [--variants bf16]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/sec, batched VELO GNN pipeline at 1 MI355X (FP32 vs BF16/FP8)"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}   # dense MFMA, MI355X
PEAK_HBM_GBS = 8000.0
STATE_BYTES = {"fp32": 4, "bf16": 2, "fp8": 2}
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def edge_net_work(H, prec, n_edges, n_hits):
    """Algorithmic work of one edge-network launch (non-final message-passing step).

    flops: two layers per edge, 3H -> H and H -> H, 2 flops per multiply-add.
    bytes: the edge state read and written once, its two hit indices, and
    every hit state read once.
    """
    s = STATE_BYTES[prec]
    flops = 2 * (3 * H * H + H * H) * n_edges
    nbytes = (2 * H * s + 8) * n_edges + H * s * n_hits
    return flops, nbytes


def roofline(stages, H, prec, n_edges, n_hits):
    ms, n = stages["edge_net"]
    if not n:
        return None
    avg_ms = ms / n
    flops, nbytes = edge_net_work(H, prec, n_edges, n_hits)
    ridge = PEAK_TFLOPS[prec] * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops / nbytes >= ridge:
        achieved = flops / (avg_ms * 1e-3) / 1e12
        return {"kernel": f"edge network ({prec} MFMA)", "bound": "mfma", "achieved": round(achieved, 3),
                "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[prec], 4),
                "traffic": None, "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops,
                "bytes_per_launch": nbytes, "arith_intensity": round(flops / nbytes, 1)}
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    return {"kernel": f"edge network ({prec} MFMA)", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops, "bytes_per_launch": nbytes,
            "arith_intensity": round(flops / nbytes, 1),
            "mfma_frac": round(flops / (avg_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec], 4)}


def run_batched(velo, synth, torch, wl, batch, hits, blob, prec, steps, warmup):
    import numpy as np
    r2 = float(np.float32(wl.radius * wl.radius))
    mx = batch.max_event_hits()
    if prec == "fp8":
        mx = max(mx, synth.calibration_batch(wl, 16).max_event_hits())
    ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, prec,
                       max_hits=batch.n_hits, max_events=batch.n_events, max_event_hits=mx)
    ctx.set_params(torch.from_numpy(blob).cuda())
    if prec == "fp8":
        calib = synth.calibration_batch(wl, 16)
        log(f"fp8: calibrating on {calib.n_events} events")
        ctx.calibrate(velo.DeviceHits.from_batch(calib))
    out = ctx.alloc_outputs(hits)
    log(f"{prec}: warmup {warmup}")
    for _ in range(warmup):
        ctx.infer(hits, out, check=False)
    ctx.check()
    n_edges = int(out["n_edges"].cpu()[0])
    ctx.set_timing(True)
    ctx.read_timing()
    torch.cuda.synchronize()
    log(f"{prec}: timing {steps} steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.infer(hits, out, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.read_timing()
    ctx.set_timing(False)
    ctx.check()
    res = {"value": round(batch.n_events * steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 4),
           "hits_per_s": round(batch.n_hits * steps / dt, 1), "edges": n_edges,
           "stage_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items()},
           "roofline": roofline(stages, wl.hidden, prec, n_edges, batch.n_hits)}
    log(f"{prec}: {res['ms_per_step']:.3f} ms/step, {res['value']:.1f} events/s")
    return ctx, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch256")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--variants", default="bf16,fp8",
                    help="comma list of extra precisions timed in the same run ('' for none)")
    ap.add_argument("--cpu-sample-events", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-event", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: events are independent, so the path shards by events "
              "with no exchange; multi-GPU runs are not part of this build (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_12119_amd import synth, velo

    wl = synth.WORKLOADS[args.workload]
    log(f"generating {wl.n_events} events ({wl.name})")
    batch = synth.make_batch(wl)
    blob = synth.centred_params(wl)
    torch.cuda.set_device(0)
    hits = velo.DeviceHits.from_batch(batch)

    ctx, main_res = run_batched(velo, synth, torch, wl, batch, hits, blob, args.precision, args.steps,
                                args.warmup)
    variants = {}
    for prec in [p for p in args.variants.split(",") if p and p != args.precision]:
        vctx, vres = run_batched(velo, synth, torch, wl, batch, hits, blob, prec, args.steps, args.warmup)
        vctx.close()
        variants[prec] = vres

    per_event = None
    if not args.no_per_event and wl.hidden <= 64:
        log("plain per-event float32 path (one call per event)")
        pctx = ctx if args.precision == "fp32" else velo.Context(
            wl.hidden, wl.iters, float(np.float32(wl.radius * wl.radius)), wl.k_max, wl.edge_logit_min, "fp32",
            max_hits=batch.n_hits, max_events=batch.n_events, max_event_hits=batch.max_event_hits())
        pctx.set_params(torch.from_numpy(blob).cuda())
        evh = [velo.DeviceHits.from_batch(synth.to_batch([batch.event(b)])) for b in range(batch.n_events)]
        outs = [pctx.alloc_outputs(h, edge_capacity=max(1, wl.k_max * h.n_hits)) for h in evh]
        for h, o in zip(evh[:8], outs[:8]):
            pctx.infer(h, o, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for h, o in zip(evh, outs):
            pctx.infer(h, o, check=False)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        pctx.check()
        per_event = {"events_per_s": round(batch.n_events / pdt, 2), "ms_total": round(1e3 * pdt, 3),
                     "precision": "fp32", "what": "the same events, one velo_infer call per event, no batching"}
        per_event["batched_speedup"] = {p: round(r["value"] / per_event["events_per_s"], 2)
                                        for p, r in [(args.precision, main_res), *variants.items()]}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        S = min(args.cpu_sample_events, batch.n_events)
        sample = synth.to_batch([batch.event(b) for b in range(S)])
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"cpu oracle on {S} events, {threads} threads")
        t0 = time.perf_counter()
        oracle.pipeline(sample, blob, wl.hidden, wl.iters, wl.radius, wl.k_max, wl.edge_logit_min)
        cdt = time.perf_counter() - t0
        cpu = {"value": round(S / cdt, 3), "unit": "events/s", "cores": threads, "kind": "oracle",
               "sample": f"first {S} events of {wl.name} ({sample.n_hits} hits), whole path, "
                         f"float64 oracle, OpenMP over events, {cdt:.1f} s"}

    recipe = wl.recipe
    comp = (f"1 vertex x {recipe.fixed_tracks} tracks" if recipe.fixed_tracks else
            f"Poisson({recipe.mu_vertices:g}) vertices x Poisson({recipe.mu_tracks:g}) tracks")
    res = {"metric": METRIC, "value": main_res["value"], "unit": "events/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision], "data": "synthetic",
           "config": {"workload": f"{wl.name}: {batch.n_events} synthetic VELO events ({comp}, "
                                  f"{recipe.noise_frac:.0%} noise), H={wl.hidden}, n={wl.iters}, "
                                  f"r={wl.radius}, k_max={wl.k_max}",
                      "events": batch.n_events, "hits": batch.n_hits, "edges": main_res["edges"],
                      "precision": args.precision},
           "hits_per_s": main_res["hits_per_s"],
           "stage_ms_per_step": main_res["stage_ms_per_step"],
           "roofline": main_res["roofline"], "cpu_baseline": cpu, "per_event_path": per_event,
           "variants": variants}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
