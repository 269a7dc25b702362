"""Training form of the edge classifier: torch.autograd bindings of the
library's forward-with-checkpoints and hand-written backward, and a small
trainer that fits the GNN on generated events.

The GNN is trained with the weighted binary cross-entropy on edge logits (the
paper trains the classifier on the same edges with a focal loss, GNN section;
the weighted BCE is this implementation's loss).  Truth labels of an edge are 1
when both hits belong to the same particle and the destination is that
particle's next hit.  The embedding MLP is not trained here: the graph is built
once per batch with the current embedding parameters and kept fixed.

Both Functions run only the library's kernels; torch supplies memory, the
stream and the autograd tape.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import synth, velo


def _torch():
    import torch
    return torch


class _EdgeLogits:
    """Holder for the lazily created autograd.Function classes (torch is
    imported on first use)."""
    fn = None
    bce = None
    focal = None


def _functions():
    if _EdgeLogits.fn is not None:
        return _EdgeLogits.fn, _EdgeLogits.bce
    torch = _torch()

    class EdgeLogits(torch.autograd.Function):
        """z = GNN(params; hits, graph) for the first n edges of `graph`.
        Backward runs velo_train_backward on the checkpoints of this forward;
        another train_forward on the same context in between is an error."""

        @staticmethod
        def forward(fctx, params, vctx, hits, graph, n):
            vctx.train_forward(hits, graph, params)
            fctx.vctx, fctx.hits, fctx.gen = vctx, hits, vctx._train_gen
            fctx.save_for_backward(params)
            return graph["edge_logit"][:n].clone()

        @staticmethod
        def backward(fctx, dz):
            (params,) = fctx.saved_tensors
            if fctx.vctx._train_gen != fctx.gen:
                raise RuntimeError("EdgeLogits.backward: the context ran another forward since this one; "
                                   "its checkpoints are gone")
            dp = fctx.vctx.train_backward(fctx.hits, params, dz.contiguous())
            return dp, None, None, None, None

    class WeightedBCE(torch.autograd.Function):
        """L = (1/n) sum_e w_e [softplus(z_e) - y_e z_e], w = pos_weight for
        y = 1 and 1 for y = 0; dL/dz from the same kernel."""

        @staticmethod
        def forward(fctx, z, vctx, y, pos_weight):
            loss, dz = vctx.bce(z.contiguous(), y, pos_weight, z.shape[0])
            fctx.save_for_backward(dz[:z.shape[0]])
            return loss[0]

        @staticmethod
        def backward(fctx, g):
            (dz,) = fctx.saved_tensors
            return dz * g, None, None, None

    class FocalLoss(torch.autograd.Function):
        """Sigmoid focal loss (the classifier loss of the GNN section):
        L = (1/n) sum_e a_t (1 - p_t)^gamma ce_e; dL/dz from the same kernel."""

        @staticmethod
        def forward(fctx, z, vctx, y, alpha, gamma):
            loss, dz = vctx.focal(z.contiguous(), y, alpha, gamma, z.shape[0])
            fctx.save_for_backward(dz[:z.shape[0]])
            return loss[0]

        @staticmethod
        def backward(fctx, g):
            (dz,) = fctx.saved_tensors
            return dz * g, None, None, None, None

    _EdgeLogits.fn, _EdgeLogits.bce, _EdgeLogits.focal = EdgeLogits, WeightedBCE, FocalLoss
    return EdgeLogits, WeightedBCE


def edge_logits(vctx: "velo.Context", params, hits: "velo.DeviceHits", graph, n_edges: int):
    """Differentiable edge logits (autograd through the library's backward)."""
    return _functions()[0].apply(params, vctx, hits, graph, n_edges)


def weighted_bce(vctx: "velo.Context", z, y, pos_weight: float):
    """Differentiable weighted BCE of logits z against uint8 labels y."""
    return _functions()[1].apply(z, vctx, y, float(pos_weight))


def focal_loss(vctx: "velo.Context", z, y, alpha: float = 0.25, gamma: float = 2.0):
    """Differentiable sigmoid focal loss of logits z against uint8 labels y."""
    _functions()
    return _EdgeLogits.focal.apply(z, vctx, y, float(alpha), float(gamma))


class GraphBatch:
    """A batch whose hits and rough graph are resident on the device, with the
    truth label of every edge."""

    def __init__(self, vctx: "velo.Context", batch: "synth.Batch"):
        torch = _torch()
        self.batch = batch
        self.hits = velo.DeviceHits.from_batch(batch)
        self.graph = vctx.build_graph(self.hits, vctx.embed(self.hits))
        g = velo.graph_to_host(self.graph)
        self.n_edges = g["n_edges"]
        ys = []
        for b in range(batch.n_events):
            s, e = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
            ys.append(synth.truth_labels(batch.event(b).next_hit, g["src"][s:e], g["dst"][s:e]))
        y = np.concatenate(ys) if ys else np.zeros(0, np.uint8)
        self.n_pos = int(y.sum())
        self.y = torch.from_numpy(y).to(self.hits.x.device)


class Trainer:
    """Adam on the GNN parameters of a float32 blob, one step per batch, with
    the library's forward, loss, backward and optimizer kernels.

    pos_weight = #negatives / #positives over the training batches, computed
    once and frozen."""

    def __init__(self, wl: "synth.Workload", params, batches: Sequence["synth.Batch"], lr: float = 3e-3):
        torch = _torch()
        self.wl = wl
        mx = max(b.max_event_hits() for b in batches)
        mh = max(b.n_hits for b in batches)
        me = max(b.n_events for b in batches)
        self.vctx = velo.Context(wl.hidden, wl.iters, float(np.float32(wl.radius * wl.radius)), wl.k_max,
                                 wl.edge_logit_min, "fp32", max_hits=mh, max_events=me, max_event_hits=mx,
                                 training=True)
        self.params = params
        self.vctx.set_params(params)
        self.data: List[GraphBatch] = [GraphBatch(self.vctx, b) for b in batches]
        n_pos = sum(d.n_pos for d in self.data)
        n_all = sum(d.n_edges for d in self.data)
        self.pos_weight = float(np.float32((n_all - n_pos) / max(n_pos, 1)))
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.lr = lr
        self.step_no = 0

    def step(self, which: Optional[int] = None):
        """One Adam step on batch `which` (round robin if None); returns the
        loss as a device tensor."""
        d = self.data[self.step_no % len(self.data) if which is None else which]
        self.vctx.train_forward(d.hits, d.graph, self.params)
        loss, dz = self.vctx.bce(d.graph["edge_logit"], d.y, self.pos_weight, d.n_edges)
        grad = self.vctx.train_backward(d.hits, self.params, dz)
        self.step_no += 1
        self.vctx.adam_step(self.params, grad, self.m, self.v, self.step_no, lr=self.lr)
        return loss

    def close(self):
        self.vctx.close()
