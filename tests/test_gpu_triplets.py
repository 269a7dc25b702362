"""GPU: the triplet stage (Sec. 5.3 triplet building and classification,
Sec. 5.4 track building) against the float64 oracle.

Stage by stage on the GPU's own upstream results, so each contract is exact
or has a stated tolerance:
  * triplet lists from the GPU's edge decisions: identical (pairs, types,
    order, per-event offsets);
  * triplet logits against the oracle's classifiers on the oracle's final
    edge encodings of the GPU's graph: |dz| <= 1e-4 * max(|z|, 1) in float32
    (the same bound as the edge logits, which come from the same encodings),
    and the bf16 bound of the edge logits with bf16 operands;
  * segments and tracks from the GPU's edge and triplet decisions: identical.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                           # noqa: E402
from paper_2407_12119_amd import synth, velo           # noqa: E402

pytestmark = pytest.mark.gpu

U = 2.0 ** -8
TRAINED = os.path.join(os.path.dirname(__file__), "golden", "trained_h64_n4.npy")
TRAINED_TRIPLETS = os.path.join(os.path.dirname(__file__), "golden", "trained_triplets_h64.npy")


def _centred_triplet_params(wl, blob, ev):
    """Seeded triplet classifiers whose output biases put the median logit of
    one event's triplets (float64 oracle) at the cut, so that about half of
    them are kept."""
    tb = synth.init_triplet_params(wl.hidden)
    emb = oracle.embed(ev.x, ev.y, ev.z, blob).astype(np.float32)
    rp, col = oracle.neighbours(ev.plane, emb, oracle.d2max_f32(wl.radius), wl.k_max)
    src, dst = oracle.csr_to_edges(rp, col)
    z, _, ef = oracle.gnn_forward(ev.x, ev.y, ev.z, src, dst, blob, wl.hidden, wl.iters, want_states=True)
    art, elb, _ = oracle.triplets(ev.n, src, dst, (z >= wl.edge_logit_min).astype(np.uint8))
    tb0 = synth.with_triplet_biases(tb, wl.hidden, 0.0, 0.0)
    ma = float(np.median(oracle.triplet_logits(art, ef, tb0, 0))) if len(art) else 0.0
    me = float(np.median(oracle.triplet_logits(elb, ef, tb0, 1))) if len(elb) else 0.0
    return synth.with_triplet_biases(tb, wl.hidden, -ma, -me)


def _run(wl, batch, blob, tblob, precision, capacity=1 << 21):
    print(f"\n[case] triplets {wl.name} {precision} events={batch.n_events} hits={batch.n_hits}", flush=True)
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, precision,
                       max_hits=max(batch.n_hits, 1), max_events=max(batch.n_events, 16),
                       max_event_hits=max(batch.max_event_hits(), 1))
    ctx.set_params(torch.from_numpy(blob).cuda())
    if precision == "fp8":
        ctx.calibrate(velo.DeviceHits.from_batch(synth.calibration_batch(wl, 4)))
    ctx.set_triplet_params(torch.from_numpy(tblob).cuda(), 0.0, capacity)
    hits = velo.DeviceHits.from_batch(batch)
    g = ctx.infer(hits)
    t = ctx.triplets(hits, g, capacity=capacity, track_capacity=capacity)
    return ctx, hits, g, t


def _check(wl, batch, blob, tblob, g, t, logit_tol):
    gh = velo.graph_to_host(g, batch.n_hits)
    th = velo.triplets_to_host(t)
    n_shared = 0
    for b in range(batch.n_events):
        ev = batch.event(b)
        s0, s1 = int(gh["edge_offsets"][b]), int(gh["edge_offsets"][b + 1])
        src, dst, z = gh["src"][s0:s1], gh["dst"][s0:s1], gh["logit"][s0:s1]
        keep = (z >= wl.edge_logit_min).astype(np.uint8)
        art, elb, et = oracle.triplets(ev.n, src, dst, keep)
        a0, a1 = int(th["art_offsets"][b]), int(th["art_offsets"][b + 1])
        e0, e1 = int(th["elb_offsets"][b]), int(th["elb_offsets"][b + 1])
        np.testing.assert_array_equal(th["art"][a0:a1], art, err_msg=f"articulations event {b}")
        np.testing.assert_array_equal(th["elb"][e0:e1], elb, err_msg=f"elbows event {b}")
        np.testing.assert_array_equal(th["elb_type"][e0:e1], et, err_msg=f"elbow types event {b}")
        za, ze = th["art_logit"][a0:a1], th["elb_logit"][e0:e1]
        if len(art) + len(elb):
            _, _, ef = oracle.gnn_forward(ev.x, ev.y, ev.z, src, dst, blob, wl.hidden, wl.iters, want_states=True)
            for zg, pairs, which in ((za, art, 0), (ze, elb, 1)):
                if len(pairs) == 0:
                    continue
                zo = oracle.triplet_logits(pairs, ef, tblob, which)
                tol = logit_tol(zo)
                err = np.abs(zg - zo)
                assert np.all(err <= tol), (b, which, float((err / tol).max()))
        ak = (za >= 0.0).astype(np.uint8)
        ek = (ze >= 0.0).astype(np.uint8)
        seg, tracks = oracle.build_tracks(ev.n, src, dst, ev.plane, keep, art, ak, elb, ek)
        np.testing.assert_array_equal(th["edge_seg"][s0:s1], seg, err_msg=f"segments event {b}")
        k0, k1 = int(th["track_offsets"][b]), int(th["track_offsets"][b + 1])
        np.testing.assert_array_equal(th["tracks"][k0:k1].reshape(-1, 2), tracks.reshape(-1, 2),
                                      err_msg=f"tracks event {b}")
        n_shared += int(np.sum(tracks[:, 1] >= 0)) if len(tracks) else 0
    print(f"  {th['n_art']} articulations ({np.mean(th['art_logit'] >= 0):.3f} kept), {th['n_elb']} elbows "
          f"({np.mean(th['elb_logit'] >= 0):.3f} kept), {th['n_tracks']} tracks, {n_shared} from shared "
          f"articulations", flush=True)
    return th, n_shared


def test_triplets_fp32_against_the_oracle():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=2, first=3)
    blob = synth.centred_params(wl)
    tblob = _centred_triplet_params(wl, blob, batch.event(0))
    ctx, hits, g, t = _run(wl, batch, blob, tblob, "fp32")
    th, n_shared = _check(wl, batch, blob, tblob, g, t, lambda z: 1e-4 * np.maximum(np.abs(z), 1.0))
    assert n_shared > 0           # shared articulations are exercised
    # bitwise repeatable, and the fused-free edge classifier gives the
    # inference logits of a context without the stage
    g2 = ctx.infer(hits)
    t2 = ctx.triplets(hits, g2, capacity=t["capacity"], track_capacity=t["track_capacity"])
    th2 = velo.triplets_to_host(t2)
    for k in ("art", "elb", "art_logit", "elb_logit", "edge_seg", "tracks"):
        np.testing.assert_array_equal(th[k], th2[k], err_msg=k)


def test_triplets_bf16_against_the_oracle():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=2, first=3)
    blob = synth.centred_params(wl)
    tblob = _centred_triplet_params(wl, blob, batch.event(0))
    # bf16 operands in the GNN and the classifier: the edge-logit bound of
    # the bf16 tests, with one more layer of depth
    _, _, g, t = _run(wl, batch, blob, tblob, "bf16")
    _check(wl, batch, blob, tblob, g, t, lambda z: (wl.iters + 3) * U + 4 * U * np.abs(z))


def test_triplets_on_trained_weights():
    if not os.path.exists(TRAINED):
        pytest.skip("trained weights not generated")
    wl = synth.WORKLOADS["batch256_trained"]
    blob = np.load(TRAINED)
    batch = synth.make_batch(wl, n_events=8, first=20)
    tblob = _centred_triplet_params(wl, blob, batch.event(0))
    _, _, g, t = _run(wl, batch, blob, tblob, "fp32")
    _check(wl, batch, blob, tblob, g, t, lambda z: 1e-4 * np.maximum(np.abs(z), 1.0))


def test_trained_triplet_classifiers_against_the_oracle():
    """The triplet classifiers trained by the oracle on the trained network's
    encodings (tests/golden/make_trained_triplets.py), float32: logits
    within 1e-4 max(|z|, 1) of the oracle's on the GPU's graph; lists,
    segments and tracks exact from the GPU's decisions."""
    if not (os.path.exists(TRAINED) and os.path.exists(TRAINED_TRIPLETS)):
        pytest.skip("trained weights not generated")
    wl = synth.WORKLOADS["batch256_trained"]
    blob = np.load(TRAINED)
    tblob = np.load(TRAINED_TRIPLETS)
    batch = synth.make_batch(wl, n_events=8, first=40)
    _, _, g, t = _run(wl, batch, blob, tblob, "fp32")
    th, _ = _check(wl, batch, blob, tblob, g, t, lambda z: 1e-4 * np.maximum(np.abs(z), 1.0))
    assert th["n_art"] > 0 and 0.5 < float(np.mean(th["art_logit"] >= 0)) < 1.0


def test_triplets_empty_events_overflow_and_order_of_calls():
    wl = synth.WORKLOADS["batch256"]
    evs = synth.make_events(wl, 2, first=3)
    empty = synth.Event(*(np.zeros(0, dt) for dt in (np.float32, np.float32, np.float32, np.int32, np.int64,
                                                      np.int32)))
    batch = synth.to_batch([empty, evs[0], empty, evs[1], empty])
    blob = synth.centred_params(wl)
    tblob = _centred_triplet_params(wl, blob, evs[0])
    ctx, hits, g, t = _run(wl, batch, blob, tblob, "fp32")
    th, _ = _check(wl, batch, blob, tblob, g, t, lambda z: 1e-4 * np.maximum(np.abs(z), 1.0))
    na, ne = th["n_art"], th["n_elb"]
    # a list that does not fit: the totals are reported, VELO_ERR_CAPACITY,
    # and the context recovers
    g = ctx.infer(hits)
    small = ctx.alloc_triplet_outputs(hits, g, 1000, 1000)
    with pytest.raises(velo.VeloError) as ei:
        ctx.triplets(hits, g, out=small)
    assert ei.value.status == velo.VELO_ERR_CAPACITY
    assert [int(v) for v in small["n_triplets"].cpu()] == [na, ne]
    # too few track slots: lists and segments written, tracks not
    g = ctx.infer(hits)
    few = ctx.alloc_triplet_outputs(hits, g, 1 << 21, 3)
    with pytest.raises(velo.VeloError) as ei:
        ctx.triplets(hits, g, out=few)
    assert ei.value.status == velo.VELO_ERR_CAPACITY
    assert int(few["n_tracks"].cpu()[0]) == th["n_tracks"]
    # the stage must directly follow the GNN pass on the same hits and graph
    g = ctx.infer(hits)
    ctx.embed(hits)
    with pytest.raises(velo.VeloError) as ei:
        ctx.triplets(hits, g)
    assert ei.value.status == velo.VELO_ERR_INVALID_ARG
    # every edge rejected: no triplets, no segments, no tracks
    cut = synth.with_classifier_bias(blob, wl.hidden, wl.iters, -1e4)
    ctx.set_params(torch.from_numpy(cut).cuda())
    g = ctx.infer(hits)
    tz = velo.triplets_to_host(ctx.triplets(hits, g, capacity=1 << 21, track_capacity=1 << 21))
    assert tz["n_art"] == 0 and tz["n_elb"] == 0 and tz["n_tracks"] == 0
    n = velo.graph_to_host(g)["n_edges"]
    assert np.all(tz["edge_seg"][:n] == -1)
