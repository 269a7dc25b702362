"""Throughput mode with several streams on one GPU, as the paper runs its
pipeline inside a multi-stream trigger framework (Sec. 7.1): every stream has
its own library context and its own share of the events, and runs them in GNN
batches whose hits and edges stay under fixed caps (the paper caps a batch at
2^20 hits and 2^22 edges).  Host-side orchestration only: every step runs in
the library's kernels, issued asynchronously on each stream.
"""
from typing import List, Sequence

import numpy as np

from . import synth, velo


def split_events(events: Sequence[synth.Event], hit_cap: int, edge_cap: int, k_max: int) -> List[synth.Batch]:
    """Consecutive runs of events as batches whose hits stay within hit_cap
    and whose edge bound (k_max per hit) within edge_cap."""
    cap = min(hit_cap, edge_cap // k_max)
    runs, cur, n = [], [], 0
    for ev in events:
        if ev.n > cap:
            raise ValueError(f"an event of {ev.n} hits exceeds the batch cap of {cap} hits")
        if cur and n + ev.n > cap:
            runs.append(cur)
            cur, n = [], 0
        cur.append(ev)
        n += ev.n
    if cur:
        runs.append(cur)
    return [synth.to_batch(r) for r in runs]


class MultiStream:
    """n_streams streams, each with a context sized for its batches and the
    device copies of its events; run() issues every stream's batches."""

    def __init__(self, wl: synth.Workload, blob: np.ndarray, precision: str,
                 events_per_stream: Sequence[Sequence[synth.Event]], hit_cap: int = 1 << 20,
                 edge_cap: int = 1 << 22):
        import torch
        r2 = float(np.float32(wl.radius * wl.radius))
        params = torch.from_numpy(blob).cuda()
        self.streams, self.ctx, self.hits, self.outs, self.batches = [], [], [], [], []
        for events in events_per_stream:
            batches = split_events(events, hit_cap, edge_cap, wl.k_max)
            mh = max(b.n_hits for b in batches)
            mx = max(b.max_event_hits() for b in batches)
            if precision == "fp8":
                calib = synth.calibration_batch(wl, 16)
                mh, mx = max(mh, calib.n_hits), max(mx, calib.max_event_hits())
            ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, precision, max_hits=mh,
                               max_events=max(max(b.n_events for b in batches), 16), max_event_hits=mx)
            ctx.set_params(params)
            if precision == "fp8":
                ctx.calibrate(velo.DeviceHits.from_batch(calib))
            hits = [velo.DeviceHits.from_batch(b) for b in batches]
            self.streams.append(torch.cuda.Stream())
            self.ctx.append(ctx)
            self.hits.append(hits)
            self.outs.append([ctx.alloc_outputs(h) for h in hits])
            self.batches.append(batches)
        torch.cuda.synchronize()

    @property
    def n_events(self) -> int:
        return sum(b.n_events for bs in self.batches for b in bs)

    def run(self):
        """Issue every stream's batches (asynchronous; call synchronize())."""
        import torch
        for s, ctx, hits, outs in zip(self.streams, self.ctx, self.hits, self.outs):
            with torch.cuda.stream(s):
                for h, o in zip(hits, outs):
                    ctx.infer(h, o, check=False)

    def synchronize(self):
        import torch
        torch.cuda.synchronize()
        for s, ctx in zip(self.streams, self.ctx):
            with torch.cuda.stream(s):
                ctx.check()

    def close(self):
        for ctx in self.ctx:
            ctx.close()
