#!/usr/bin/env python3
"""Throughput of the batched VELO GNN track-finding path on one MI355X.

One step = one call of the whole path (embedding, rough graph, GNN, edge cut,
components) over one batch of synthetic events already resident in HBM.
Prints ONE JSON line (rank 0) with events/s, the roofline of the dominant
kernel measured with HIP events over the timed region, the float64 CPU oracle
timed on a bounded sample of the same workload, and the plain per-event path.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch256]
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def edge_net_flops_per_edge(H):
    # two layers per edge: 3H -> H and H -> H, 2 flops per multiply-add
    return 2 * (3 * H * H + H * H)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch256")
    ap.add_argument("--precision", default="fp32", choices=["fp32"])
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
    r2 = float(np.float32(wl.radius * wl.radius))
    torch.cuda.set_device(0)
    hits = velo.DeviceHits.from_batch(batch)
    ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, args.precision,
                       max_hits=batch.n_hits, max_events=batch.n_events,
                       max_event_hits=batch.max_event_hits())
    ctx.set_params(torch.from_numpy(blob).cuda())
    out = ctx.alloc_outputs(hits)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.infer(hits, out, check=False)
    ctx.check()
    n_edges = int(out["n_edges"].cpu()[0])

    ctx.set_timing(True)
    ctx.read_timing()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.infer(hits, out, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.read_timing()
    ctx.set_timing(False)
    ctx.check()
    ms_step = 1e3 * dt / args.steps
    ev_s = batch.n_events / (dt / args.steps)
    hits_s = batch.n_hits / (dt / args.steps)
    log(f"{ms_step:.3f} ms/step, {ev_s:.1f} events/s")

    # dominant kernel: the edge network (non-final steps), an MFMA contraction
    H = wl.hidden
    ms_en, n_en = stages["edge_net"]
    roof = None
    if n_en:
        avg_ms = ms_en / n_en
        flops = edge_net_flops_per_edge(H) * n_edges
        achieved = flops / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": "edge network (k_mlp EDGE, MFMA 16x16x4 f32)", "bound": "mfma",
                "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[args.precision], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[args.precision], 4), "traffic": None,
                "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops,
                "flops_per_edge": edge_net_flops_per_edge(H)}

    per_event = None
    if not args.no_per_event:
        log("plain per-event path (one call per event)")
        evh = [velo.DeviceHits.from_batch(synth.to_batch([batch.event(b)])) for b in range(batch.n_events)]
        outs = [ctx.alloc_outputs(h, edge_capacity=max(1, wl.k_max * h.n_hits)) for h in evh]
        for h, o in zip(evh[:8], outs[:8]):
            ctx.infer(h, o, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for h, o in zip(evh, outs):
            ctx.infer(h, o, check=False)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        ctx.check()
        per_event = {"events_per_s": round(batch.n_events / pdt, 2),
                     "ms_total": round(1e3 * pdt, 3), "precision": "fp32",
                     "what": "the same events, one velo_infer call per event, no batching"}

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

    res = {"metric": METRIC, "value": round(ev_s, 2), "unit": "events/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[args.precision],
           "data": "synthetic",
           "config": {"workload": f"{wl.name}: {batch.n_events} synthetic pile-up events "
                                  f"(Poisson(5) vertices x Poisson(30) tracks), H={wl.hidden}, "
                                  f"n={wl.iters}, r={wl.radius}, k_max={wl.k_max}",
                      "events": batch.n_events, "hits": batch.n_hits, "edges": n_edges,
                      "precision": args.precision},
           "hits_per_s": round(hits_s, 1),
           "stage_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
           "roofline": roof, "cpu_baseline": cpu, "per_event_path": per_event}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
