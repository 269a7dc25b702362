"""Pins of the oracle's embedding training (Sec. 5.1, the two loss equations):
the pair sets against a brute-force enumeration written here from the text,
the gradient against central finite differences of the float64 loss, and
two cases the mathematics fixes (a constant embedding; translation
invariance of squared distances)."""
import numpy as np
import pytest

import oracle
from paper_2407_12119_amd import synth

WL = synth.WORKLOADS["batch256"]
E0 = 12                                   # first embedding entry of the blob
NE = 128 * 3 + 128 + 128 * 128 + 128 + 4 * 128 + 4
B3 = E0 + NE - 4                          # the output bias (4 entries)


def _event(n_keep=None, seed=0):
    tb = synth.embed_train_batch(synth.make_events(WL, 1, first=seed), step=seed)
    ev = tb.batch.event(0)
    n = ev.n if n_keep is None else n_keep
    # keep the first n hits (still sorted by plane)
    return (ev.x[:n], ev.y[:n], ev.z[:n], ev.plane[:n], tb.pid[:n], tb.query[:n], tb.rnd[:n])


def _sums(ev, blob, emb32, **kw):
    x, y, z, plane, pid, query, rnd = ev
    return oracle.embed_train_sums(x, y, z, plane, pid, query, rnd, emb32, blob, **kw)


def _d2_f32(a, b):
    # float32 squared distance in the order d0*d0, then fma(d_c, d_c, s);
    # each product of two float32 values is exact in float64
    d = (a[0] - b[0]).astype(np.float32)
    s = np.float32(np.float64(d) * np.float64(d))
    for c in range(1, 4):
        d = np.float32(a[c] - b[c])
        s = np.float32(np.float64(d) * np.float64(d) + np.float64(s))
    return s


def test_pair_sets_match_brute_force():
    ev = _event(n_keep=120, seed=3)
    x, y, z, plane, pid, query, rnd = ev
    blob = synth.init_params(WL)
    e64 = oracle.embed(x, y, z, blob)
    e32 = e64.astype(np.float32)
    k_train, d2_train = 7, np.float32(1.5)
    n = x.shape[0]
    pairs = []
    for q in range(n):
        if not query[q]:
            continue
        cands = [j for j in range(n) if plane[j] - plane[q] in (1, 2)]
        near = sorted((float(_d2_f32(e32[q], e32[j])), j) for j in cands)
        near = [j for d, j in near if d < d2_train][:k_train]
        pairs += [(q, j) for j in sorted(near) if pid[j] != pid[q]]          # hard negatives
        pairs += [(q, j) for j in cands if pid[j] == pid[q]]                 # genuine
        if cands:
            pairs.append((q, cands[(int(rnd[q]) * len(cands)) >> 32]))       # random
    # a margin inside the fake pairs' distances, so that some hinges are off
    fake_d2 = [float(_d2_f32(e32[q], e32[j])) for q, j in pairs if pid[j] != pid[q]]
    margin = float(np.float32(np.median(fake_d2)))
    Sg = Sf = 0.0
    Ng = Nf = off = 0
    for q, j in pairs:
        d2 = float(np.sum((e64[q] - e64[j]) ** 2))
        if pid[j] == pid[q]:
            Ng += 1
            Sg += d2
        else:
            Nf += 1
            if _d2_f32(e32[q], e32[j]) < np.float32(margin):
                Sf += margin - d2
            else:
                off += 1
    assert 0 < off < Nf
    sg, sf, ng, nf, _, _ = _sums(ev, blob, e32, k_train=k_train, d2_train=float(d2_train), margin=margin)
    assert (ng, nf) == (Ng, Nf)
    assert ng > 10 and nf > 10
    assert sg == pytest.approx(Sg, rel=1e-12)
    assert sf == pytest.approx(Sf, rel=1e-12)


def test_gradient_matches_finite_differences():
    ev = _event(n_keep=160, seed=1)
    x, y, z = ev[0], ev[1], ev[2]
    blob = synth.init_params(WL)
    # the decisions (neighbour list, active hinges) stay those of the
    # unperturbed float32 embedding, so the loss is smooth in the parameters
    e32 = oracle.embed(x, y, z, blob).astype(np.float32)
    w = 3.0

    def loss(b):
        return oracle.embed_train_loss([_sums(ev, b, e32)], w)

    base = loss(blob)
    assert base["n_genuine"] > 0 and base["n_fake"] > 0
    g = base["grad"]
    rng = np.random.default_rng(5)
    segs = [(E0, 384), (E0 + 384, 128), (E0 + 512, 16384), (E0 + 16896, 128), (E0 + 17024, 512)]
    idx = [int(o + rng.integers(0, m)) for o, m in segs for _ in range(3)]
    idx += [int(E0 + 17024 + np.argmax(np.abs(g[E0 + 17024:E0 + 17536])))]
    h = 2.0 ** -12
    scale = np.abs(g[E0:E0 + NE]).max()
    for q in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[q] += np.float32(h)
        bm[q] -= np.float32(h)
        fd = (loss(bp)["loss"] - loss(bm)["loss"]) / (float(bp[q]) - float(bm[q]))
        assert fd == pytest.approx(g[q], abs=2e-5 * scale), q


def test_constant_embedding_gives_the_margin_and_no_gradient():
    # W1 = W2 = 0: every hit has the same embedding, every d2 is 0, so the
    # genuine term is 0, every fake pair's hinge is active with value m, and
    # L = m exactly with a zero gradient
    ev = _event(n_keep=200, seed=2)
    x, y, z = ev[0], ev[1], ev[2]
    blob = synth.init_params(WL)
    blob[E0:E0 + 384] = 0.0
    blob[E0 + 512:E0 + 512 + 16384] = 0.0
    e32 = oracle.embed(x, y, z, blob).astype(np.float32)
    assert np.all(e32 == e32[0])
    r = oracle.embed_train_loss([_sums(ev, blob, e32, margin=1.0)], 2.0)
    assert r["n_fake"] > 0
    assert r["loss"] == 1.0 and r["loss_genuine"] == 0.0
    assert np.all(r["grad"] == 0.0)


def test_output_bias_gradient_vanishes():
    # squared distances do not change when every embedding moves by the same
    # vector: dL/db3 = 0 exactly in exact arithmetic
    parts = []
    blob = synth.init_params(WL)
    for seed in (4, 5):
        ev = _event(n_keep=250, seed=seed)
        e32 = oracle.embed(ev[0], ev[1], ev[2], blob).astype(np.float32)
        parts.append(_sums(ev, blob, e32, k_train=20, d2_train=2.0))
    r = oracle.embed_train_loss(parts, 2.0)
    scale = np.abs(r["grad"][E0:E0 + NE]).max()
    assert scale > 0
    assert np.abs(r["grad"][B3:B3 + 4]).max() <= 1e-12 * scale
