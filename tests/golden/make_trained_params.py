"""Write trained_h64_n4.npy: a trained network (embedding and GNN) made by the
float64 oracle alone, for the tests that compare the low-precision paths with
the oracle on trained weights, and for the benchmark's quality block.

The seeded random init keeps nearly every logit close to the cut and every
activation small; trained weights are larger and their logits decisive,
which is where bf16/fp8 rounding shows.  Training uses only oracle/
(gradients in float64) and numpy (Adam), on generated events of their own
seed stream, so no value here comes from the GPU path.

  1. Embedding (Sec. 5.1): pairwise hinge loss over hard negatives from the
     bounded neighbour list (k = 50, d^2 < 1.5), genuine pairs and one random
     pair per query hit, on noise-free events, margin 1, w_genuine = 2;
     Adam (lr 1e-3) on the embedding entries.
  2. GNN (Sec. 5.2): weighted BCE on the rough graph of the trained
     embedding at the paper's inference values (d^2 < 0.9, k_max = 50), on
     events with noise; truth = consecutive hits of one particle; pos_weight
     = #neg / #pos of the training events, frozen; Adam with a cosine
     learning-rate decay 3e-3 -> 3e-5 on the GNN entries.

Run:  python tests/golden/make_trained_params.py   (about 10 minutes, 8 threads)
"""
import hashlib
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle                                        # noqa: E402
from paper_2407_12119_amd import synth              # noqa: E402

OUT = os.path.join(HERE, "trained_h64_n4.npy")
LOG = os.path.join(HERE, "trained_h64_n4.json")

WL = synth.WORKLOADS["batch256_trained"]
EMB_K, EMB_D2, EMB_M, EMB_WG = 50, 1.5, 1.0, 2.0
EMB_STEPS, EMB_EVENTS, EMB_LR = 300, 4, 1e-3
GNN_STEPS, GNN_EVENTS, GNN_LR0, GNN_LR1 = 300, 8, 3e-3, 3e-5
POOL = 32                       # training events (seed stream synth.TRAINED_TRAIN_INDEX)
THREADS = 8


class Adam:
    """Kingma and Ba's Adam with bias correction, float64 state, on a slice."""

    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, p, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - lr * mh / (np.sqrt(vh) + self.eps)


def emb_slice():
    n_norm = 12
    n_emb = sum(o * i + o for name, (o, i) in synth.param_layout(WL.hidden, WL.iters) if name.startswith("emb"))
    return slice(n_norm, n_norm + n_emb)


def train_embedding(blob, events, pool):
    sl = emb_slice()
    p = blob[sl].astype(np.float64)
    opt = Adam(p.size)
    curve = []
    for step in range(EMB_STEPS):
        chosen = [events[(step * EMB_EVENTS + i) % len(events)] for i in range(EMB_EVENTS)]
        tb = synth.embed_train_batch(chosen, step=step)
        off = tb.batch.event_offsets
        cur = blob.copy()
        cur[sl] = p.astype(np.float32)

        def one(e):
            a, b = int(off[e]), int(off[e + 1])
            ev = tb.batch.event(e)
            emb32 = oracle.embed(ev.x, ev.y, ev.z, cur).astype(np.float32)
            return oracle.embed_train_sums(ev.x, ev.y, ev.z, ev.plane, tb.pid[a:b], tb.query[a:b], tb.rnd[a:b],
                                           emb32, cur, EMB_K, EMB_D2, EMB_M)

        parts = list(pool.map(one, range(len(chosen))))
        res = oracle.embed_train_loss(parts, EMB_WG)
        p = opt.step(p, res["grad"][sl], EMB_LR)
        curve.append(res["loss"])
        if step % 25 == 0 or step == EMB_STEPS - 1:
            print(f"embedding step {step}: loss {res['loss']:.4f}", flush=True)
    blob = blob.copy()
    blob[sl] = p.astype(np.float32)
    return blob, curve


def graph_of(ev, blob):
    emb32 = oracle.embed(ev.x, ev.y, ev.z, blob).astype(np.float32)
    rp, col = oracle.neighbours(ev.plane, emb32, oracle.d2max_f32(WL.radius), WL.k_max)
    src, dst = oracle.csr_to_edges(rp, col)
    return src, dst, synth.truth_labels(ev.next_hit, src, dst)


def train_gnn(blob, events, pool):
    graphs = list(pool.map(lambda ev: graph_of(ev, blob), events))
    n_pos = sum(int(g[2].sum()) for g in graphs)
    n_all = sum(g[2].size for g in graphs)
    pos_weight = float(np.float32((n_all - n_pos) / max(n_pos, 1)))
    true_total = sum(int((ev.next_hit >= 0).sum()) for ev in events)
    print(f"training graphs: {n_all} edges on {sum(ev.n for ev in events)} hits, {n_pos} true "
          f"({n_pos / max(true_total, 1):.4f} of the consecutive-hit pairs); pos_weight {pos_weight:.3f}",
          flush=True)
    sl = slice(emb_slice().stop, blob.size)
    p = blob[sl].astype(np.float64)
    opt = Adam(p.size)
    curve = []
    for step in range(GNN_STEPS):
        idx = [(step * GNN_EVENTS + i) % len(events) for i in range(GNN_EVENTS)]
        cur = blob.copy()
        cur[sl] = p.astype(np.float32)
        z = list(pool.map(lambda i: oracle.gnn_forward(events[i].x, events[i].y, events[i].z, graphs[i][0],
                                                       graphs[i][1], cur, WL.hidden, WL.iters), idx))
        sizes = np.cumsum([0] + [zz.size for zz in z])
        L, dz = oracle.bce(np.concatenate(z), np.concatenate([graphs[i][2] for i in idx]), pos_weight)
        grads = pool.map(lambda k: oracle.gnn_backward(events[idx[k]].x, events[idx[k]].y, events[idx[k]].z,
                                                       graphs[idx[k]][0], graphs[idx[k]][1], cur, WL.hidden,
                                                       WL.iters, dz[sizes[k]:sizes[k + 1]]), range(len(idx)))
        g = sum(grads)
        lr = GNN_LR1 + 0.5 * (GNN_LR0 - GNN_LR1) * (1 + math.cos(math.pi * step / GNN_STEPS))
        p = opt.step(p, g[sl], lr)
        curve.append(float(L))
        if step % 25 == 0 or step == GNN_STEPS - 1:
            print(f"gnn step {step}: loss {L:.4f}", flush=True)
    blob = blob.copy()
    blob[sl] = p.astype(np.float32)
    return blob, curve, pos_weight


def main():
    t0 = time.time()
    oracle.set_threads(1)
    events = [synth.make_event(WL.recipe, synth.event_rng(synth.TRAINED_TRAIN_INDEX, e)) for e in range(POOL)]
    blob = synth.init_params(WL)
    with ThreadPoolExecutor(THREADS) as pool:
        blob, emb_curve = train_embedding(blob, events, pool)
        blob, gnn_curve, pos_weight = train_gnn(blob, events, pool)
    np.save(OUT, blob)
    digest = hashlib.sha256(blob.tobytes()).hexdigest()
    log = {"what": "embedding and GNN trained by the float64 oracle (see the script's docstring)",
           "workload": WL.name, "hidden": WL.hidden, "iters": WL.iters, "d2_max": oracle.d2max_f32(WL.radius),
           "k_max": WL.k_max, "training_events": f"{POOL} events of seed stream {synth.TRAINED_TRAIN_INDEX}",
           "embedding": {"steps": EMB_STEPS, "events_per_step": EMB_EVENTS, "lr": EMB_LR, "k_train": EMB_K,
                         "d2_train": EMB_D2, "margin": EMB_M, "w_genuine": EMB_WG,
                         "loss_first": emb_curve[0], "loss_last10_mean": float(np.mean(emb_curve[-10:]))},
           "gnn": {"steps": GNN_STEPS, "events_per_step": GNN_EVENTS, "lr": f"cosine {GNN_LR0} -> {GNN_LR1}",
                   "pos_weight": pos_weight, "loss_first": gnn_curve[0],
                   "loss_last10_mean": float(np.mean(gnn_curve[-10:]))},
           "sha256_float32_blob": digest, "seconds": round(time.time() - t0, 1)}
    with open(LOG, "w") as f:
        json.dump(log, f, indent=1)
    print(json.dumps(log, indent=1), flush=True)


if __name__ == "__main__":
    main()
