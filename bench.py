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
                       [--precision fp32|bf16|bf16x2|fp8] [--variants bf16,bf16x2,fp8] [--no-graph] [--latency]
       the 1000-event workload: --workload batch1000_h128 --precision bf16 --variants fp8
                                --latency --no-cpu-baseline
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/sec, batched VELO GNN pipeline at 1 MI355X (FP32 vs BF16/FP8)"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2, "bf16x2": 2516.6}   # dense MFMA, MI355X
PEAK_HBM_GBS = 8000.0
STATE_BYTES = {"fp32": 4, "bf16": 2, "fp8": 2, "bf16x2": 2}
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8", "bf16x2": "bf16x2"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def edge_net_work(H, prec, n_edges, n_hits):
    """Algorithmic work of one edge-network launch (non-final message-passing step).

    bf16/fp8 (concatenated first layer): two layers per edge, 3H -> H and
    H -> H, 2 flops per multiply-add; bytes: the edge state read and written
    once, its two hit indices, every hit state read once, and the float32
    outgoing message sum of every hit (H floats) written.
    fp32 (factorised first layer): the hit segments' products come from the
    per-hit projection (timed as its own stage), so per edge the launch does
    the e segment of the first layer (H -> H) and the second layer; bytes:
    the edge state read and written once, its two hit indices and every
    hit's pair of float32 products (2H floats) read once.
    """
    s = STATE_BYTES[prec]
    if s == 4:
        flops = 2 * (H * H + H * H) * n_edges
        nbytes = (2 * H * s + 8) * n_edges + 2 * H * 4 * n_hits
        return flops, nbytes
    flops = 2 * (3 * H * H + H * H) * n_edges
    nbytes = (2 * H * s + 8) * n_edges + H * s * n_hits + 4 * H * n_hits
    return flops, nbytes


def copy_probe_gbs(torch, mib=1024, reps=10):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of a
    plain `copy_` of `mib` MiB: what a streaming kernel reaches on this GPU."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "edge_net_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2407_12119_amd", "csrc", f) for f in ("gnn.hip", "mfma.h", "internal.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(prec, workload):
    """HBM bytes per edge-network launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if it was taken on the current kernel
    source and this workload; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(prec)
    if not e or t.get("source_sha1") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def stage_roofline(stages, steps, H, iters, prec, N, E):
    """Per-stage roofline of one step (one pass of the whole path): for each
    group of stages, the algorithmic flops F and HBM bytes B of the method
    (not of this implementation), T_roof = max(F / MFMA peak, B / HBM peak),
    the measured time T and T_roof / T.  s = bytes per stored encoding
    element; messages are float32 in every precision.  F is the method's
    cheapest exact form: a first layer over concatenated hit encodings
    [h_i; h_j] is W_s h_i + W_d h_j, with the products taken once per hit
    (2 H^2 flops per hit and segment) and only the edge's own segment per
    edge; the 2-byte paths multiply the concatenation per edge instead, which
    is more matrix work for the same result.
      embedding       F = 34,560 N                 B = 28 N (inputs, embedding)
      graph           F = 0 (integer/ALU)          B = 24 N + 16 E (embedding read, row pointers and
                                                   the event-local edge pairs out; incoming lists 8 E + 4 N)
      encoders        F = 2(3H + H^2) N + 4 H^2 N + 2 H^2 E
                                                   B = 12 N + s H N + (s H + 8) E
      message passing F = n (12 H^2 N + 4 H^2 E) + 2 (H^2 + H) E (with the classifier)
                      B = n ((2 s H + 8) E + (2 s H + 16 H) N) + 4 E
      components      F = 0                        B = 9 E + 16 N
    The float32 path's per-hit first-layer products (hit_proj) count with
    message passing."""
    s = STATE_BYTES[prec]
    P = PEAK_TFLOPS[prec] * 1e12
    BW = PEAK_HBM_GBS * 1e9
    groups = {
        "embedding": (["embed"], 34560 * N, 28 * N),
        "graph": (["prepare", "knn", "compact", "lists"], 0, 24 * N + 16 * E),
        "encoders": (["node_enc", "edge_enc"], 2 * (3 * H + H * H) * N + 4 * H * H * N + 2 * H * H * E,
                     12 * N + s * H * N + (s * H + 8) * E),
        "message_passing": (["hit_proj", "messages", "node_net", "edge_net", "edge_cls"],
                            iters * (12 * H * H * N + 4 * H * H * E) + 2 * (H * H + H) * E,
                            iters * ((2 * s * H + 8) * E + (2 * s * H + 16 * H) * N) + 4 * E),
        "components": (["components"], 0, 9 * E + 16 * N),
    }
    out, tr, tm = {}, 0.0, 0.0
    for name, (keys, F, B) in groups.items():
        t = sum(stages.get(k, (0.0, 0))[0] for k in keys) / steps
        roof = max(F / P, B / BW) * 1e3
        out[name] = {"t_ms": round(t, 4), "t_roof_ms": round(roof, 4), "frac": round(roof / t, 4) if t > 0 else None,
                     "bound": "mfma" if F / P > B / BW else "hbm", "flops": int(F), "bytes": int(B),
                     "achieved_GBps": round(B / (t * 1e-3) / 1e9, 1) if t > 0 else None}
        if F:
            out[name]["achieved_TFLOPs"] = round(F / (t * 1e-3) / 1e12, 2) if t > 0 else None
        tr += roof
        tm += t
    out["total"] = {"t_ms": round(tm, 4), "t_roof_ms": round(tr, 4), "frac": round(tr / tm, 4) if tm > 0 else None}
    return out


def roofline(stages, H, prec, n_edges, n_hits, workload, copy_gbs=None):
    ms, n = stages["edge_net"]
    if not n:
        return None
    avg_ms = ms / n
    flops, nbytes = edge_net_work(H, prec, n_edges, n_hits)
    if STATE_BYTES[prec] == 4 and stages.get("hit_proj", (0.0, 0))[1]:
        # the float32 edge network's hit segments are multiplied per hit by
        # hit_proj: its launches (one per edge MLP) are part of the work
        hp_ms, hp_n = stages["hit_proj"]
        proj = hp_ms / hp_n
        achieved = (flops + 4 * H * H * n_hits) / ((avg_ms + proj) * 1e-3) / 1e12
        concat = 2 * (3 * H * H + H * H) * n_edges / ((avg_ms + proj) * 1e-3) / 1e12
        return {"kernel": "edge network with its per-hit first-layer products (fp32 MFMA)", "bound": "mfma",
                "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[prec], 4), "traffic": measured_traffic(prec, workload),
                "avg_launch_ms": round(avg_ms, 4), "hit_proj_ms": round(proj, 4),
                "flops_per_launch": flops + 4 * H * H * n_hits, "bytes_per_launch": nbytes,
                "arith_intensity": round(flops / nbytes, 1),
                "frac_of_concatenated_count": round(concat / PEAK_TFLOPS[prec], 4)}
    ridge = PEAK_TFLOPS[prec] * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops / nbytes >= ridge:
        achieved = flops / (avg_ms * 1e-3) / 1e12
        return {"kernel": f"edge network ({prec} MFMA)", "bound": "mfma", "achieved": round(achieved, 3),
                "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[prec], 4),
                "traffic": measured_traffic(prec, workload), "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops,
                "bytes_per_launch": nbytes, "arith_intensity": round(flops / nbytes, 1)}
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    res = {"kernel": f"edge network ({prec} MFMA)", "bound": "hbm", "achieved": round(achieved, 1),
           "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
           "traffic": measured_traffic(prec, workload),
           "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops, "bytes_per_launch": nbytes,
           "arith_intensity": round(flops / nbytes, 1),
           "mfma_frac": round(flops / (avg_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec], 4)}
    if copy_gbs:
        res["copy_frac"] = round(achieved / copy_gbs, 4)
    return res


def run_training(velo, synth, torch, steps, warmup):
    """Training step of the 32-event workload (H = 64, n = 6, fp32): forward with
    checkpoints, weighted BCE, backward, Adam.  Graph building is the input
    pipeline and stays outside the timed region."""
    import numpy as np
    wl = synth.WORKLOADS["train32"]
    batch = synth.make_batch(wl)
    blob = synth.init_params(wl)
    ctx = velo.Context(wl.hidden, wl.iters, float(np.float32(wl.radius * wl.radius)), wl.k_max,
                       wl.edge_logit_min, "fp32", max_hits=batch.n_hits, max_events=batch.n_events,
                       max_event_hits=batch.max_event_hits(), training=True)
    params = torch.from_numpy(blob).cuda()
    ctx.set_params(params)
    hits = velo.DeviceHits.from_batch(batch)
    graph = ctx.build_graph(hits, ctx.embed(hits))
    g = velo.graph_to_host(graph, batch.n_hits)
    ys = [synth.truth_labels(batch.event(b).next_hit, g["src"][g["edge_offsets"][b]:g["edge_offsets"][b + 1]],
                             g["dst"][g["edge_offsets"][b]:g["edge_offsets"][b + 1]]) for b in range(batch.n_events)]
    y = np.concatenate(ys)
    pw = float((y == 0).sum()) / max(float(y.sum()), 1.0)
    yt = torch.from_numpy(y).cuda()
    n = g["n_edges"]
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    grad = torch.empty_like(params)

    def step(t):
        ctx.train_forward(hits, graph, params)
        _, dz = ctx.bce(graph["edge_logit"], yt, pw, n)
        ctx.train_backward(hits, params, dz, grad)
        ctx.adam_step(params, grad, m, v, t, lr=1e-3)

    for t in range(1, warmup + 1):
        step(t)
    ctx.set_timing(True)
    ctx.read_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup + 1, warmup + steps + 1):
        step(t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.read_timing()
    ctx.set_timing(False)
    ctx.check()
    log(f"training: {1e3 * dt / steps:.3f} ms/step")
    return {"workload": f"{wl.name}: {batch.n_events} events, {batch.n_hits} hits, {n} edges, H={wl.hidden}, "
                        f"n={wl.iters}, fp32, weighted BCE (pos_weight {pw:.2f}), Adam",
            "steps_per_s": round(steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 3),
            "stage_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items() if v[1]}}


EMB_TRAIN = {"k_train": 50, "d2_train": 1.5, "margin": 1.0, "w_genuine": 2.0}   # Sec. 5.1 (w: a reading)


def run_embed_training(velo, synth, torch, steps, warmup, train_steps):
    """Embedding training step (Sec. 5.1) on 32 noise-free events: loss and
    gradient (pairs, hinge loss, back-propagation) and Adam on the embedding
    entries.  Then, when train_steps > 0, train_steps steps over four such
    batches and the rough graph (d2 < 0.9, k = 50: the paper's inference
    values) of 32 other events with noise, before and after."""
    import numpy as np
    wl = synth.WORKLOADS["train32"]
    tbs = [synth.embed_train_batch(synth.make_events(wl, 32, first=32 * i), step=i) for i in range(4)]
    cap = max(tb.batch.n_hits for tb in tbs)
    ctx = velo.Context(wl.hidden, wl.iters, float(np.float32(wl.radius * wl.radius)), wl.k_max,
                       wl.edge_logit_min, "fp32", max_hits=cap, max_events=32,
                       max_event_hits=max(tb.batch.max_event_hits() for tb in tbs), training=True)
    blob = synth.init_params(wl)
    params = torch.from_numpy(blob).cuda()
    ctx.set_params(params)
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).cuda()
    data = [(velo.DeviceHits.from_batch(tb.batch), dev(tb.pid, np.int32), dev(tb.query, np.uint8),
             dev(tb.rnd.view(np.int32), np.int32)) for tb in tbs]
    sl = slice(12, 12 + 17540)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    grad = torch.zeros_like(params)
    losses = []

    def step(t, d, keep=False):
        _, loss, _ = ctx.embed_train_grad(*d, params, dparams=grad, **EMB_TRAIN)
        ctx.adam_step(params[sl], grad[sl], m[sl], v[sl], t, lr=1e-3)
        if keep:
            losses.append(loss)

    for t in range(1, warmup + 1):
        step(t, data[0])
    ctx.set_timing(True)
    ctx.read_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup + 1, warmup + steps + 1):
        step(t, data[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.read_timing()
    ctx.set_timing(False)
    ctx.check()
    n0 = tbs[0].batch.n_hits
    log(f"embedding training: {1e3 * dt / steps:.3f} ms/step")
    res = {"workload": f"embed_train32: 32 noise-free events, {n0} hits, k_train={EMB_TRAIN['k_train']}, "
                       f"d2_train={EMB_TRAIN['d2_train']}, m={EMB_TRAIN['margin']}, "
                       f"w_genuine={EMB_TRAIN['w_genuine']}, fp32, Adam",
           "steps_per_s": round(steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 3),
           "stage_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items() if v[1]}}
    if train_steps <= 0:
        return res

    # rough graph of 32 held-out events (with noise) at the paper's inference values
    ev_batch = synth.make_batch(synth.WORKLOADS["batch256"], 32, first=1000)
    gctx = velo.Context(wl.hidden, wl.iters, 0.9, 50, wl.edge_logit_min, "fp32",
                        max_hits=ev_batch.n_hits, max_events=32, max_event_hits=ev_batch.max_event_hits())
    ehits = velo.DeviceHits.from_batch(ev_batch)

    def graph_stats(p):
        gctx.set_params(p)
        g = velo.graph_to_host(gctx.build_graph(ehits, gctx.embed(ehits)), ev_batch.n_hits)
        true_total = found = 0
        for b in range(ev_batch.n_events):
            ev = ev_batch.event(b)
            s, e = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
            have = set(zip(g["src"][s:e].tolist(), g["dst"][s:e].tolist()))
            nh = ev.next_hit
            for i in np.flatnonzero(nh >= 0):
                if ev.plane[nh[i]] - ev.plane[i] in (1, 2):
                    true_total += 1
                    found += (int(i), int(nh[i])) in have
        E = int(g["n_edges"])
        return {"edges_per_hit": round(E / max(ev_batch.n_hits, 1), 2),
                "true_edge_recall": round(found / max(true_total, 1), 4)}

    before = graph_stats(torch.from_numpy(blob).cuda())
    params.copy_(torch.from_numpy(blob).cuda())
    m.zero_(); v.zero_()
    losses.clear()
    t0 = time.perf_counter()
    for t in range(1, train_steps + 1):
        step(t, data[(t - 1) % 4], keep=(t <= 4 or t > train_steps - 4))
    torch.cuda.synchronize()
    ttrain = time.perf_counter() - t0
    after = graph_stats(params)
    gctx.close()
    ls = [float(x[0].cpu()) for x in losses]
    res["training_run"] = {"steps": train_steps, "seconds": round(ttrain, 2),
                           "loss_first": round(float(np.mean(ls[:4])), 5), "loss_last": round(float(np.mean(ls[-4:])), 5),
                           "rough_graph_d2_0.9_k50": {"init": before, "trained": after}}
    log(f"embedding training run: {json.dumps(res['training_run'])}")
    return res


TRAINED_BLOB = os.path.join(ROOT, "tests", "golden", "trained_h64_n4.npy")


def run_quality(velo, synth, torch, precisions):
    """Track-finding quality at every precision with a trained network: the
    embedding and GNN trained by the float64 oracle on generated events of
    their own seed stream (tests/golden/make_trained_params.py), run on the
    256 benchmark events with the paper's inference values of the rough
    graph (d^2 < 0.9, k_max = 50).  Each lower precision is compared with
    fp32: end to end (its own embedding, so its own graph: decisions over
    the union of the two edge sets, Jaccard overlap, largest logit
    difference on common edges) and on the fp32 graph (the GNN's own
    error)."""
    import numpy as np
    from paper_2407_12119_amd import metrics
    if not os.path.exists(TRAINED_BLOB):
        return {"skipped": "trained weights not generated"}
    wl = synth.WORKLOADS["batch256_trained"]
    blob = np.load(TRAINED_BLOB)
    batch = synth.make_batch(wl)
    hits = velo.DeviceHits.from_batch(batch)
    r2 = float(np.float32(wl.radius * wl.radius))
    res, ref, ref_dev = {}, None, None
    for prec in precisions:
        mx = batch.max_event_hits()
        if prec == "fp8":
            mx = max(mx, synth.calibration_batch(wl, 16).max_event_hits())
        ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, prec, max_hits=batch.n_hits,
                           max_events=batch.n_events, max_event_hits=mx)
        ctx.set_params(torch.from_numpy(blob).cuda())
        if prec == "fp8":
            ctx.calibrate(velo.DeviceHits.from_batch(synth.calibration_batch(wl, 16)))
        dev = ctx.infer(hits)
        g = velo.graph_to_host(dev, batch.n_hits)
        m = metrics.track_metrics(g["labels"], batch.pid, batch.event_offsets)
        r = {k: round(m[k], 5) for k in ("efficiency", "clone_rate", "fake_rate", "hit_efficiency", "hit_purity")}
        r["edges"] = g["n_edges"]
        r["edges_per_hit"] = round(g["n_edges"] / batch.n_hits, 3)
        r["kept_edges"] = int((g["logit"] >= wl.edge_logit_min).sum())
        if ref is None:
            ref = g
            ref_dev = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in dev.items()}
            true_kept = 0
            for b in range(batch.n_events):
                s0, s1 = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
                true_kept += int(synth.truth_labels(batch.event(b).next_hit, g["src"][s0:s1], g["dst"][s0:s1]).sum())
            r["true_edges_in_graph"] = round(true_kept / max(int((batch.next_hit >= 0).sum()), 1), 5)
        else:
            a = metrics.edge_agreement(ref["edge_offsets"], ref["src"], ref["dst"], ref["logit"] >= wl.edge_logit_min,
                                       g["edge_offsets"], g["src"], g["dst"], g["logit"] >= wl.edge_logit_min)
            r["d_efficiency_pts"] = round(100 * (m["efficiency"] - res[precisions[0]]["efficiency"]), 4)
            r["decision_agreement"] = round(a["decision_agreement"], 6)
            r["jaccard"] = round(a["jaccard"], 6)
            gs = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in ref_dev.items()}
            ctx.gnn(hits, gs)
            ctx.components(hits, gs)
            same = velo.graph_to_host(gs, batch.n_hits)
            zr = ref["logit"].astype(np.float64)
            dz = np.abs(same["logit"] - zr) / np.maximum(np.abs(zr), 1.0)
            ms = metrics.track_metrics(same["labels"], batch.pid, batch.event_offsets)
            r["on_fp32_graph"] = {
                "max_logit_err": round(float(dz.max()), 6) if dz.size else 0.0,
                "p99_logit_err": round(float(np.percentile(dz, 99)), 6) if dz.size else 0.0,
                "decision_agreement": round(float(np.mean((same["logit"] >= wl.edge_logit_min) ==
                                                          (ref["logit"] >= wl.edge_logit_min))), 6),
                "d_efficiency_pts": round(100 * (ms["efficiency"] - res[precisions[0]]["efficiency"]), 4)}
        ctx.close()
        res[prec] = r
    # the INT8 embedding (Sec. 7.4, Table 5: INT8 adds a few percent of edges),
    # calibrated on 16 other events, with the rest of the path in float32
    cal = synth.calibration_batch(wl, 16)
    ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, "fp32",
                       max_hits=max(batch.n_hits, cal.n_hits), max_events=max(batch.n_events, cal.n_events),
                       max_event_hits=max(batch.max_event_hits(), cal.max_event_hits()))
    ctx.set_params(torch.from_numpy(blob).cuda())
    ctx.calibrate_embed_int8(velo.DeviceHits.from_batch(cal))
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    ctx.close()
    m = metrics.track_metrics(g["labels"], batch.pid, batch.event_offsets)
    a = metrics.edge_agreement(ref["edge_offsets"], ref["src"], ref["dst"], ref["logit"] >= wl.edge_logit_min,
                               g["edge_offsets"], g["src"], g["dst"], g["logit"] >= wl.edge_logit_min)
    res["int8_embedding"] = {"edges": g["n_edges"], "extra_edges_frac": round(g["n_edges"] / ref["n_edges"] - 1.0, 5),
                             "jaccard": round(a["jaccard"], 6), "decision_agreement": round(a["decision_agreement"], 6),
                             "efficiency": round(m["efficiency"], 5),
                             "d_efficiency_pts": round(100 * (m["efficiency"] - res[precisions[0]]["efficiency"]), 4),
                             "what": "INT8 embedding (calibrated on 16 other events), float32 GNN, against fp32"}
    res["triplets"] = run_triplet_quality(velo, torch, wl, batch, hits, blob, r2)
    res["weights"] = "trained by the float64 oracle (embedding 300 steps, GNN 300 steps; see trained_h64_n4.json)"
    res["workload"] = f"{wl.name}: the {batch.n_events} benchmark events, d2 < 0.9, k_max = {wl.k_max}"
    log(f"quality: {json.dumps(res)}")
    return res


TRAINED_TRIPLETS = os.path.join(ROOT, "tests", "golden", "trained_triplets_h64.npy")


def run_triplet_quality(velo, torch, wl, batch, hits, blob, r2, reps=10):
    """The triplet stage (Sec. 5.3, 5.4) on the benchmark batch with the
    trained network and the triplet classifiers trained by the oracle on its
    final edge encodings (tests/golden/make_trained_triplets.py): tracks
    built from the purified edge graph against the connected components of
    the purified hit graph (the paper's with and without triplets), and the
    stage's time per batch (triplet building, both classifiers, track
    building), with the classifiers' matrix work."""
    import numpy as np
    from paper_2407_12119_amd import metrics
    if not os.path.exists(TRAINED_TRIPLETS):
        return {"skipped": "trained triplet classifiers not generated"}
    tb = np.load(TRAINED_TRIPLETS)
    keys = ("efficiency", "clone_rate", "fake_rate", "hit_efficiency", "hit_purity")
    out = {"classifiers": "trained by the float64 oracle (see trained_triplets_h64.json)"}
    for prec in ("fp32", "bf16x2"):
        ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, prec, max_hits=batch.n_hits,
                           max_events=batch.n_events, max_event_hits=batch.max_event_hits())
        ctx.set_params(torch.from_numpy(blob).cuda())
        ctx.set_triplet_params(torch.from_numpy(tb).cuda(), 0.0, 1 << 22)
        g = ctx.infer(hits)
        t = ctx.triplets(hits, g)
        ctx.set_timing(True)
        ctx.read_timing()
        for _ in range(reps):
            ctx.triplets(hits, g, out=t, check=False)
        ms = ctx.read_timing()["triplets"][0] / reps
        ctx.set_timing(False)
        ctx.check()
        gh, th = velo.graph_to_host(g, batch.n_hits), velo.triplets_to_host(t)
        tracks = []
        for b in range(batch.n_events):
            s0, s1 = int(gh["edge_offsets"][b]), int(gh["edge_offsets"][b + 1])
            k0, k1 = int(th["track_offsets"][b]), int(th["track_offsets"][b + 1])
            tracks.append(metrics.track_hit_lists(gh["src"][s0:s1], gh["dst"][s0:s1], th["edge_seg"][s0:s1],
                                                  th["tracks"][k0:k1]))
        mt = metrics.track_list_metrics(tracks, batch.pid, batch.event_offsets)
        mw = metrics.track_metrics(gh["labels"], batch.pid, batch.event_offsets)
        H = wl.hidden
        n_tri = th["n_art"] + th["n_elb"]
        flops = n_tri * 2 * (2 * H * H + H)        # hidden layer [2H -> H] and output [H -> 1] per triplet
        out[prec] = {"with_triplets": {k: round(mt[k], 5) for k in keys},
                     "without_triplets": {k: round(mw[k], 5) for k in keys},
                     "d_efficiency_pts": round(100 * (mt["efficiency"] - mw["efficiency"]), 3),
                     "articulations": th["n_art"], "articulations_kept": round(float(np.mean(th["art_logit"] >= 0)), 4),
                     "elbows": th["n_elb"], "elbows_kept": round(float(np.mean(th["elb_logit"] >= 0)), 4)
                     if th["n_elb"] else 0.0,
                     "tracks": th["n_tracks"], "stage_ms": round(ms, 4),
                     "classifier_gflop": round(flops / 1e9, 3),
                     "classifier_tflops_over_stage": round(flops / (ms * 1e-3) / 1e12, 3) if ms > 0 else None}
        log(f"triplets {prec}: {json.dumps(out[prec])}")
        ctx.close()
    return out


def transfer_times(torch, batch, out, n_edges, reps=5):
    """Host-device copies around one batch, outside the timed region: the hit
    arrays to the device and labels, edge pairs and logits back, with pinned
    host buffers (median of a few repetitions)."""
    import numpy as np
    host = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
            for a in (batch.event_offsets.astype(np.int32), batch.x, batch.y, batch.z, batch.plane.astype(np.int32))]
    dev = [torch.empty_like(h, device="cuda") for h in host]
    srcs = [out["labels"][:batch.n_hits], out["edge_src"][:n_edges], out["edge_dst"][:n_edges],
            out["edge_logit"][:n_edges], out["edge_offsets"]]
    back = [torch.empty(t.shape, dtype=t.dtype, pin_memory=True) for t in srcs]
    h2d, d2h = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d, h in zip(dev, host):
            d.copy_(h, non_blocking=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for b, d in zip(back, srcs):
            b.copy_(d, non_blocking=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        h2d.append(t1 - t0)
        d2h.append(t2 - t1)
    nb_in = sum(h.numel() * h.element_size() for h in host)
    nb_out = sum(b.numel() * b.element_size() for b in back)
    return {"h2d_ms": round(1e3 * float(np.median(h2d)), 4), "h2d_bytes": nb_in,
            "d2h_ms": round(1e3 * float(np.median(d2h)), 4), "d2h_bytes": nb_out}


def sweep_compare(ctx, torch, hits, reps=10):
    """The paper's plane-sweep components (Sec. 7.3; a comparison variant)
    against the exact components on the same decisions: the time of each
    components stage and the share of hits the sweep labels differently."""
    out = ctx.infer(hits)
    exact = out["labels"].clone()
    times = {}
    for name, fn in (("exact", ctx.components), ("sweep", ctx.components_sweep)):
        fn(hits, out)
        ctx.set_timing(True)
        ctx.read_timing()
        for _ in range(reps):
            fn(hits, out, check=False)
        torch.cuda.synchronize()
        times[name] = round(ctx.read_timing()["components"][0] / reps, 4)
        ctx.set_timing(False)
    differ = int((out["labels"][:hits.n_hits] != exact[:hits.n_hits]).sum().cpu())
    ctx.check()
    return {"exact_ms": times["exact"], "sweep_ms": times["sweep"], "hits": hits.n_hits,
            "hits_labelled_differently": differ, "fraction": round(differ / max(hits.n_hits, 1), 5)}


def knn_compare(ctx, torch, hits, reps=5):
    """The paper's per-hit neighbour loop (Sec. 7.2; a comparison variant)
    against the wavefront search, on the same embedding: neighbour-search
    stage time of each and whether the graphs agree."""
    emb = ctx.embed(hits)
    times, graphs = {}, {}
    for name, fn in (("wavefront", ctx.build_graph), ("paper_loop", ctx.build_graph_loop)):
        out = fn(hits, emb)
        ctx.set_timing(True)
        ctx.read_timing()
        for _ in range(reps):
            fn(hits, emb, out=out, check=False)
        torch.cuda.synchronize()
        times[name] = round(ctx.read_timing()["knn"][0] / reps, 4)
        ctx.set_timing(False)
        n = int(out["n_edges"].cpu()[0])
        graphs[name] = (out["edge_dst"][:n].clone(), out["edge_offsets"].clone())
    ctx.check()
    same = bool(torch.equal(graphs["wavefront"][0], graphs["paper_loop"][0]) and
                torch.equal(graphs["wavefront"][1], graphs["paper_loop"][1]))
    return {"wavefront_ms": times["wavefront"], "paper_loop_ms": times["paper_loop"],
            "speedup": round(times["paper_loop"] / max(times["wavefront"], 1e-9), 2), "same_graph": same}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_agreement(synth, wl, sample, ref, gpu):
    """The GPU path's results on the sampled events against the float64
    oracle's (from raw hits, end to end): edge sets (Jaccard), decisions
    over the union of the two edge sets, the largest logit difference
    |z - z_oracle| / max(|z_oracle|, 1) on common edges, identical labels,
    and the track-finding efficiency difference in points."""
    import numpy as np
    from paper_2407_12119_amd import metrics
    S, n = sample.n_events, sample.n_hits
    E = int(gpu["edge_offsets"][S])
    g = {"off": gpu["edge_offsets"][:S + 1], "src": gpu["src"][:E], "dst": gpu["dst"][:E], "z": gpu["logit"][:E],
         "labels": gpu["labels"][:n]}
    cut = wl.edge_logit_min
    a = metrics.edge_agreement(ref["edge_offsets"], ref["src"], ref["dst"], ref["logit"] >= cut, g["off"], g["src"],
                               g["dst"], g["z"] >= cut)
    kr = metrics.edge_keys(ref["edge_offsets"], ref["src"], ref["dst"])
    kg = metrics.edge_keys(g["off"], g["src"], g["dst"])
    _, ia, ib = np.intersect1d(kr, kg, return_indices=True)
    zr = ref["logit"][ia]
    err = np.abs(g["z"][ib] - zr) / np.maximum(np.abs(zr), 1.0) if ia.size else np.zeros(1)
    mo = metrics.track_metrics(ref["labels"], sample.pid, sample.event_offsets)
    mg = metrics.track_metrics(g["labels"], sample.pid, sample.event_offsets)
    # the pairs in one edge set only, by the oracle's float64 embedding
    # distance: within 1e-6 relative of the radius (reported separately), at
    # the row's k_max-th distance (within 1e-5 relative: the bounded list's
    # cut), or neither
    kd = np.setxor1d(kr, kg)
    eoff = np.asarray(sample.event_offsets, np.int64)
    ev, i, j = kd >> 42, (kd >> 21) & ((1 << 21) - 1), kd & ((1 << 21) - 1)
    emb = np.asarray(ref["emb"], np.float64)
    d2 = ((emb[eoff[ev] + i] - emb[eoff[ev] + j]) ** 2).sum(1) if kd.size else np.zeros(0)
    rs = np.repeat(np.arange(S, dtype=np.int64), np.diff(np.asarray(ref["edge_offsets"], np.int64)))
    ref_d2 = ((emb[eoff[rs] + ref["src"]] - emb[eoff[rs] + ref["dst"]]) ** 2).sum(1)
    row_key = (rs << 21) | np.asarray(ref["src"], np.int64)
    kth = {}
    if row_key.size:
        order = np.argsort(row_key, kind="stable")
        keys, first, counts = np.unique(row_key[order], return_index=True, return_counts=True)
        mx = np.maximum.reduceat(ref_d2[order], first)
        kth = {int(k): float(m) for k, m, c in zip(keys, mx, counts) if c >= wl.k_max}
    near_r = int(np.sum(np.abs(np.sqrt(d2) - wl.radius) <= 1e-6 * wl.radius))
    at_k = 0
    for e in range(kd.size):
        if abs(math.sqrt(d2[e]) - wl.radius) <= 1e-6 * wl.radius:
            continue
        dk = kth.get(int((ev[e] << 21) | i[e]))
        if dk is not None and abs(d2[e] - dk) <= 1e-5 * max(dk, 1e-12):
            at_k += 1
    return {"jaccard": round(a["jaccard"], 6), "decision_agreement": round(a["decision_agreement"], 6),
            "edges_in_one_set": int(kd.size), "of_which_within_1e-6_of_radius": near_r,
            "of_which_at_k_max_cut": at_k, "of_which_other": int(kd.size) - near_r - at_k,
            "max_logit_err": round(float(err.max()), 6), "p99_logit_err": round(float(np.percentile(err, 99)), 6),
            "labels_identical": round(float(np.mean(g["labels"] == ref["labels"])), 6),
            "efficiency_oracle": round(mo["efficiency"], 5),
            "d_efficiency_pts": round(100 * (mg["efficiency"] - mo["efficiency"]), 4)}


def run_cpu_baseline(synth, wl, batch, blob, n_sample, n_single, samples):
    """The float64 oracle timed on the host: the first n_sample events of
    the workload on all host threads (OpenMP over events), and the first
    n_single on one thread; its outputs on the sample then measure each
    GPU precision's agreement with it."""
    import oracle
    S = min(n_sample, batch.n_events)
    sample = synth.to_batch([batch.event(b) for b in range(S)])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    log(f"cpu oracle on {S} events, {threads} threads")
    t0 = time.perf_counter()
    ref = oracle.pipeline(sample, blob, wl.hidden, wl.iters, wl.radius, wl.k_max, wl.edge_logit_min)
    cdt = time.perf_counter() - t0
    S1 = min(n_single, S)
    one = synth.to_batch([batch.event(b) for b in range(S1)])
    oracle.set_threads(1)
    log(f"cpu oracle on {S1} events, 1 thread")
    t0 = time.perf_counter()
    oracle.pipeline(one, blob, wl.hidden, wl.iters, wl.radius, wl.k_max, wl.edge_logit_min)
    sdt = time.perf_counter() - t0
    oracle.set_threads(threads)
    cpu = {"value": round(S / cdt, 3), "unit": "events/s", "cores": threads, "kind": "oracle",
           "sample": f"first {S} events of {wl.name} ({sample.n_hits} hits), whole path, "
                     f"float64 oracle, OpenMP over events, {cdt:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "single_thread": {"value": round(S1 / sdt, 3), "unit": "events/s", "cores": 1,
                             "sample": f"first {S1} events ({one.n_hits} hits), {sdt:.1f} s"},
           "note": "a correctness oracle, not a tuned CPU implementation"}
    if samples:
        cpu["gpu_vs_oracle"] = {p: oracle_agreement(synth, wl, sample, ref, g) for p, g in samples.items()}
        log(f"gpu vs oracle on the sample: {json.dumps(cpu['gpu_vs_oracle'])}")
    return cpu


def run_large(velo, synth, torch, steps, warmup, autotune):
    """The 1000-event workload (Poisson(12) x Poisson(30) tracks, 10% noise;
    H = 128, n = 8) with bf16 MLP operands: eager events/s, then the whole
    path captured once into a HIP graph and replayed, with per-batch latency
    percentiles."""
    wl = synth.WORKLOADS["batch1000_h128"]
    log(f"generating {wl.n_events} events ({wl.name})")
    batch = synth.make_batch(wl)
    blob = synth.centred_params(wl)
    hits = velo.DeviceHits.from_batch(batch)
    ctx, res = run_batched(velo, synth, torch, wl, batch, hits, blob, "bf16", steps, warmup, True, True, autotune)
    ctx.close()
    res.pop("transfer", None)
    res["workload"] = (f"{wl.name}: {batch.n_events} events, {batch.n_hits} hits (up to "
                       f"{batch.max_event_hits()} per event), H={wl.hidden}, n={wl.iters}, bf16")
    del hits
    torch.cuda.empty_cache()
    return res


def run_multistream(synth, torch, wl, blob, prec, n_streams, events_per_stream, passes=3):
    """Throughput with n_streams streams on the GPU, each with its own
    context and events_per_stream events run in batches capped at 2^20 hits
    and 2^22 edges (the paper's multi-stream setting, Sec. 7.1), against one
    stream under the same caps.  Every stream gets the same events."""
    from paper_2407_12119_amd import multistream
    events = synth.make_events(wl, events_per_stream, first=3000)
    res = {"precision": prec, "events_per_stream": events_per_stream, "hit_cap": 1 << 20, "edge_cap": 1 << 22}
    for label, ns in (("one_stream", 1), ("streams", n_streams)):
        ms = multistream.MultiStream(wl, blob, prec, [events] * ns)
        ms.run()
        ms.synchronize()
        t0 = time.perf_counter()
        for _ in range(passes):
            ms.run()
        ms.synchronize()
        dt = time.perf_counter() - t0
        res[label] = {"streams": ns, "batches_per_stream": len(ms.batches[0]),
                      "events_per_s": round(ms.n_events * passes / dt, 1), "seconds": round(dt, 3)}
        ms.close()
    log(f"multi-stream: {json.dumps(res)}")
    return res


def parse_tuning(velo, text):
    """'stage=k,stage=k' -> {stage: k}, checked against the stage names and
    the candidate table."""
    choice = {}
    for item in text.split(","):
        stage, _, k = item.partition("=")
        stage = stage.strip()
        if stage not in velo.STAGES or not k.strip().isdigit() or int(k) >= len(velo.AUTOTUNE_CANDIDATES):
            raise SystemExit(f"--tuning: bad entry {item!r} (stages {', '.join(velo.STAGES)}; "
                             f"candidates 0..{len(velo.AUTOTUNE_CANDIDATES) - 1})")
        choice[stage] = int(k)
    return choice


def run_batched(velo, synth, torch, wl, batch, hits, blob, prec, steps, warmup, graph=False, latency=False,
                autotune=True, copy_gbs=None, samples=None):
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
    tuned = None
    if isinstance(autotune, dict):   # a stored choice (--tuning), applied instead of measured
        ctx.set_tuning(autotune)
        tuned = {k: autotune.get(k, 0) for k in velo.STAGES}
        log(f"{prec}: tuning {autotune}")
    log(f"{prec}: warmup {warmup}")
    for _ in range(warmup):
        ctx.infer(hits, out, check=False)
    ctx.check()
    if tuned is None and autotune:
        tuned = ctx.autotune(hits, out)
        log(f"{prec}: autotune choice {tuned}")
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
    if samples is not None:
        samples[prec] = velo.graph_to_host(out, batch.n_hits)
    res = {"value": round(batch.n_events * steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 4),
           "hits_per_s": round(batch.n_hits * steps / dt, 1), "edges": n_edges,
           "stage_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items()},
           "roofline": roofline(stages, wl.hidden, prec, n_edges, batch.n_hits, wl.name, copy_gbs),
           "stage_roofline": stage_roofline(stages, steps, wl.hidden, wl.iters, prec, batch.n_hits, n_edges)}
    # events/s of the path cut after each stage (cumulative, in path order)
    order = ["prepare", "embed", "knn", "compact", "lists", "node_enc", "hit_proj", "edge_enc", "messages",
             "node_net", "edge_net", "edge_cls", "components"]
    acc, cum = 0.0, {}
    for k in order:
        acc += res["stage_ms_per_step"].get(k, 0.0)
        if acc > 0:
            cum[k] = round(batch.n_events / (acc * 1e-3), 1)
    res["cumulative_events_per_s"] = cum
    tr = transfer_times(torch, batch, out, n_edges)
    tr["pcie_inclusive_events_per_s"] = round(batch.n_events / (1e-3 * (tr["h2d_ms"] + res["ms_per_step"] +
                                                                        tr["d2h_ms"])), 1)
    res["transfer"] = tr
    if tuned is not None:
        shape = {"knn": ("mem_per_cu", "knn_run", "xcd"), "messages": ("mem_per_cu", "xcd")}
        res["autotune"] = {k: {"candidate": v, **{f: velo.AUTOTUNE_CANDIDATES[v][f]
                                                 for f in shape.get(k, ("mlp_per_cu", "mlp_block", "xcd"))}}
                           for k, v in tuned.items() if k in ("knn", "edge_enc", "messages", "node_net",
                                                              "edge_net", "edge_cls")}
    log(f"{prec}: {res['ms_per_step']:.3f} ms/step, {res['value']:.1f} events/s")
    if graph or latency:
        # the whole path captured once into a HIP graph and replayed; per-batch
        # latency from HIP events around each replay
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            gr = ctx.capture(hits, out) if graph else None
            run = gr.launch if gr is not None else (lambda: ctx.infer(hits, out, check=False))
            for _ in range(warmup):
                run()
            side.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(steps)]
            t0 = time.perf_counter()
            for a, b in evs:
                a.record(side)
                run()
                b.record(side)
            side.synchronize()
            gdt = time.perf_counter() - t0
            lat = np.array([a.elapsed_time(b) for a, b in evs])
        ctx.check()
        key = "graph" if graph else "eager"
        res[key] = {"value": round(batch.n_events * steps / gdt, 2), "ms_per_step": round(1e3 * gdt / steps, 4),
                    "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                    "latency_ms_p99": round(float(np.percentile(lat, 99)), 4)}
        log(f"{prec} {key}: {res[key]['ms_per_step']:.3f} ms/step, p50 {res[key]['latency_ms_p50']:.3f} ms, "
            f"p99 {res[key]['latency_ms_p99']:.3f} ms")
        if gr is not None:
            gr.close()
    return ctx, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch256")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "bf16x2", "fp8"])
    ap.add_argument("--variants", default="bf16,bf16x2,fp8",
                    help="comma list of extra precisions timed in the same run ('' for none)")
    ap.add_argument("--cpu-sample-events", type=int, default=32)
    ap.add_argument("--cpu-single-events", type=int, default=4,
                    help="events of the single-thread oracle timing")
    ap.add_argument("--no-large", action="store_true", help="skip the 1000-event H = 128 bf16 block")
    ap.add_argument("--large-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-event", action="store_true")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step measurement")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the hipGraph replays of the whole path (timed beside the eager steps by default)")
    ap.add_argument("--latency", action="store_true", help="per-batch p50/p99 latency (of the hipGraph replays unless --no-graph)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in launch parameters")
    ap.add_argument("--tuning", default="",
                    help="apply this candidate choice instead of autotuning (stage=k,...; stages not named: 0), "
                         "e.g. to profile only the launches a tuned run makes")
    ap.add_argument("--no-quality", action="store_true", help="skip the track-finding quality block")
    ap.add_argument("--streams", type=int, default=16,
                    help="multi-stream throughput mode: streams (0 to skip)")
    ap.add_argument("--stream-events", type=int, default=500, help="events per stream in the multi-stream mode")
    ap.add_argument("--embed-train-steps", type=int, default=300,
                    help="embedding training steps before the rough-graph comparison (with the quality block)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a float32 add of this size (reads and writes known bytes): the reference "
                         "kernel that scales the HBM traffic counters of a profiled run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: events are independent, so the path shards by events "
              "with no exchange; multi-GPU runs are not implemented (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_12119_amd import synth, velo

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        torch.add(x, 1.0, out=y)
        torch.cuda.synchronize()
        log(f"copy probe: {4 * n} bytes read, {4 * n} bytes written")
        del x, y

    wl = synth.WORKLOADS[args.workload]
    log(f"generating {wl.n_events} events ({wl.name})")
    batch = synth.make_batch(wl)
    blob = synth.centred_params(wl)
    torch.cuda.set_device(0)
    hits = velo.DeviceHits.from_batch(batch)
    copy_gbs = copy_probe_gbs(torch)
    log(f"device copy probe: {copy_gbs} GB/s (read + write)")

    samples = {}
    tune = parse_tuning(velo, args.tuning) if args.tuning else not args.no_autotune
    ctx, main_res = run_batched(velo, synth, torch, wl, batch, hits, blob, args.precision, args.steps,
                                args.warmup, not args.no_graph, args.latency, tune, copy_gbs, samples)
    sweep = sweep_compare(ctx, torch, hits)
    log(f"components, exact vs the paper's plane sweeps: {json.dumps(sweep)}")
    knn_loop = knn_compare(ctx, torch, hits)
    log(f"neighbour search, wavefront vs the paper's per-hit loop: {json.dumps(knn_loop)}")
    variants = {}
    for prec in [p for p in args.variants.split(",") if p and p != args.precision]:
        vctx, vres = run_batched(velo, synth, torch, wl, batch, hits, blob, prec, args.steps, args.warmup,
                                 not args.no_graph, args.latency, tune, copy_gbs, samples)
        vctx.close()
        variants[prec] = vres
    multi = None
    if args.streams > 0 and args.workload == "batch256":
        multi = run_multistream(synth, torch, wl, blob, "bf16", args.streams, args.stream_events)
        # the form that meets the precision targets on trained weights
        multi["bf16x2"] = run_multistream(synth, torch, wl, blob, "bf16x2", args.streams, args.stream_events)
    training = None
    embed_training = None
    if not args.no_train and args.workload == "batch256":
        training = run_training(velo, synth, torch, max(5, args.steps // 2), 2)
        embed_training = run_embed_training(velo, synth, torch, max(5, args.steps // 2), 2,
                                            0 if args.no_quality else args.embed_train_steps)

    quality = None
    if not args.no_quality and args.workload == "batch256":
        quality = run_quality(velo, synth, torch,
                              ["fp32"] + [p for p in ("bf16", "bf16x2", "fp8") if p in [args.precision] + list(variants)])

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
        cpu = run_cpu_baseline(synth, wl, batch, blob, args.cpu_sample_events, args.cpu_single_events, samples)

    large = None
    if not args.no_large and args.workload == "batch256":
        ctx.close()
        large = run_large(velo, synth, torch, args.large_steps, 2, tune)

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
           "roofline": main_res["roofline"], "hbm_copy_GBps": copy_gbs, "cpu_baseline": cpu, "per_event_path": per_event,
           "variants": variants, "training": training, "embed_training": embed_training, "components_sweep": sweep, "knn_paper_loop": knn_loop, "multi_stream": multi, "quality": quality,
           "stage_roofline": main_res["stage_roofline"], "batch1000_h128": large}
    for k in ("graph", "eager"):
        if k in main_res:
            res[k] = main_res[k]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
