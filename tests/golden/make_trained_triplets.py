"""Write trained_triplets_h64.npy: the two triplet classifiers (Sec. 5.3)
trained by the float64 oracle on the final edge encodings of the trained
network in trained_h64_n4.npy, for the benchmark's comparison of tracks with
and without triplets (Sec. 5.4) and the GPU triplet test on trained
classifiers.  No value here comes from the GPU path.

For each training event (the network's own training events, seed stream
synth.TRAINED_TRAIN_INDEX): the rough graph of the trained embedding at the
paper's inference values (d^2 < 0.9, k_max = 50), the oracle's GNN forward
with its final edge encodings, the edges kept at logit >= 0 and the
articulations and elbows of the kept edges (oracle.triplets).  A triplet is
genuine iff both of its edges are true (consecutive hits of one particle).
The generator has no shared hits, so no elbow is genuine there and the elbow
classifier learns to reject them.

Loss: weighted binary cross-entropy per classifier (pos_weight = #negative /
#positive triplets of the pool, 1 without positives), Adam with a cosine
learning-rate decay 3e-3 -> 3e-5, gradients from
oracle.triplet_classifier_grad.  The embedding and the GNN stay fixed: the
paper trains the GNN and the triplet classifiers together on the sum of the
two losses; here the classifiers are fitted to the trained GNN's encodings.

Run:  python tests/golden/make_trained_triplets.py   (a few minutes, 8 threads)
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
sys.path.insert(0, HERE)

import oracle                                        # noqa: E402
from paper_2407_12119_amd import synth              # noqa: E402
from make_trained_params import Adam, POOL, THREADS, WL, graph_of   # noqa: E402

NET = os.path.join(HERE, "trained_h64_n4.npy")
OUT = os.path.join(HERE, "trained_triplets_h64.npy")
LOG = os.path.join(HERE, "trained_triplets_h64.json")
STEPS, EVENTS, LR0, LR1 = 300, 8, 3e-3, 3e-5


def event_triplets(ev, blob):
    """Pairs, truth and final edge encodings of one event's triplets."""
    src, dst, truth = graph_of(ev, blob)
    z, _, ef = oracle.gnn_forward(ev.x, ev.y, ev.z, src, dst, blob, WL.hidden, WL.iters, want_states=True)
    keep = (z >= WL.edge_logit_min).astype(np.uint8)
    art, elb, _ = oracle.triplets(ev.n, src, dst, keep)
    y = [(truth[p[:, 0]] & truth[p[:, 1]]).astype(np.float64) if len(p) else np.zeros(0) for p in (art, elb)]
    return {"pairs": (art, elb), "y": y, "e": ef}


def main():
    t0 = time.time()
    oracle.set_threads(1)
    blob = np.load(NET)
    H = WL.hidden
    per = 2 * H * H + 2 * H + 1
    events = [synth.make_event(WL.recipe, synth.event_rng(synth.TRAINED_TRAIN_INDEX, e)) for e in range(POOL)]
    with ThreadPoolExecutor(THREADS) as pool:
        data = list(pool.map(lambda ev: event_triplets(ev, blob), events))
        tb = synth.init_triplet_params(H).astype(np.float64)
        log = {"what": "triplet classifiers trained by the float64 oracle (see the script's docstring)",
               "network": os.path.basename(NET), "training_events": f"{POOL} events of seed stream "
                                                                     f"{synth.TRAINED_TRAIN_INDEX}",
               "steps": STEPS, "events_per_step": EVENTS, "lr": f"cosine {LR0} -> {LR1}"}
        for which, name in ((0, "articulations"), (1, "elbows")):
            n_pos = sum(int(d["y"][which].sum()) for d in data)
            n_all = sum(d["y"][which].size for d in data)
            pos_weight = float(np.float32((n_all - n_pos) / n_pos)) if n_pos else 1.0
            print(f"{name}: {n_all} triplets, {n_pos} genuine; pos_weight {pos_weight:.3f}", flush=True)
            sl = slice(which * per, (which + 1) * per)
            p = tb[sl].copy()
            opt = Adam(p.size)
            curve = []
            for step in range(STEPS):
                idx = [i % len(data) for i in range(step * EVENTS, (step + 1) * EVENTS)]
                idx = [i for i in idx if data[i]["y"][which].size]
                if not idx:
                    break
                cur = tb.copy()
                cur[sl] = p
                cur32 = cur.astype(np.float32)
                z = list(pool.map(lambda i: oracle.triplet_logits(data[i]["pairs"][which], data[i]["e"], cur32,
                                                                  which), idx))
                sizes = np.cumsum([0] + [zz.size for zz in z])
                L, dz = oracle.bce(np.concatenate(z), np.concatenate([data[i]["y"][which] for i in idx]),
                                   pos_weight)
                g = sum(pool.map(lambda k: oracle.triplet_classifier_grad(
                    data[idx[k]]["pairs"][which], data[idx[k]]["e"], cur32, which, dz[sizes[k]:sizes[k + 1]]),
                    range(len(idx))))
                lr = LR1 + 0.5 * (LR0 - LR1) * (1 + math.cos(math.pi * step / STEPS))
                p = opt.step(p, g, lr)
                curve.append(float(L))
                if step % 25 == 0 or step == STEPS - 1:
                    print(f"{name} step {step}: loss {L:.4f}", flush=True)
            tb[sl] = p
            # decisions of the trained classifier on the pool
            cur32 = tb.astype(np.float32)
            right = sum(int(((oracle.triplet_logits(d["pairs"][which], d["e"], cur32, which) >= 0) ==
                             (d["y"][which] > 0)).sum()) for d in data if d["y"][which].size)
            log[name] = {"triplets": n_all, "genuine": n_pos, "pos_weight": pos_weight,
                         "loss_first": curve[0] if curve else None,
                         "loss_last10_mean": float(np.mean(curve[-10:])) if curve else None,
                         "pool_accuracy": right / max(n_all, 1)}
    out = tb.astype(np.float32)
    np.save(OUT, out)
    log["sha256_float32_blob"] = hashlib.sha256(out.tobytes()).hexdigest()
    log["seconds"] = round(time.time() - t0, 1)
    with open(LOG, "w") as f:
        json.dump(log, f, indent=1)
    print(json.dumps(log, indent=1), flush=True)


if __name__ == "__main__":
    main()
