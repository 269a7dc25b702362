"""Pins of the oracle's triplet stage (Sec. 5.3 triplet building and
classifiers, Sec. 5.4 track building from the purified edge graph).

* Triplet lists against a brute-force enumeration over all pairs of kept
  edges that share a hit, and the closed-form counts
  sum_C in_C out_C (articulations), sum_C C(out_C, 2) and sum_C C(in_C, 2)
  (left and right elbows).
* Classifier special cases: with a zero first layer every triplet gets the
  same closed-form logit; first layers that read only one half of the input
  separate the order [e_a || e_b].
* Track building on graphs worked by hand: a chain (one track), two tracks
  that share their first hits (the articulations at the parting are shared,
  so each track gets a copy of the shared edge), a triangle with a plane-
  skipping edge (the elbows join it and mark it a duplicate, so no spurious
  sharing), and two tracks bridged by a kept fake edge whose triplets are
  rejected (three tracks where connected components give one).
* Track-list metrics equal the label metrics when tracks are components.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2407_12119_amd import metrics


def _brute_triplets(n, src, dst, keep):
    kept = [q for q in range(len(src)) if keep[q]]
    art, left, right = set(), set(), set()
    for a, b in itertools.permutations(kept, 2):
        if dst[a] == src[b]:
            art.add((a, b))
        if a < b and src[a] == src[b]:
            left.add((a, b))
        if a < b and dst[a] == dst[b]:
            right.add((a, b))
    return art, left, right


def _random_graph(rng, n=40, m=160):
    plane = np.sort(rng.integers(0, 8, n)).astype(np.int32)
    pairs = set()
    while len(pairs) < m:
        i, j = (int(v) for v in rng.integers(0, n, 2))
        if plane[j] - plane[i] in (1, 2):
            pairs.add((i, j))
    e = np.array(sorted(pairs), np.int32)
    return plane, e[:, 0].copy(), e[:, 1].copy()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_triplets_against_brute_force_and_counts(seed):
    rng = np.random.default_rng(seed)
    n = 40
    plane, src, dst = _random_graph(rng, n)
    keep = (rng.random(len(src)) < 0.7).astype(np.uint8)
    art, elb, et = oracle.triplets(n, src, dst, keep)
    b_art, b_left, b_right = _brute_triplets(n, src, dst, keep)
    assert set(map(tuple, art.tolist())) == b_art and len(art) == len(b_art)
    assert set(map(tuple, elb[et == 1].tolist())) == b_left
    assert set(map(tuple, elb[et == 2].tolist())) == b_right
    ks = keep.astype(bool)
    din = np.bincount(dst[ks], minlength=n)
    dout = np.bincount(src[ks], minlength=n)
    assert len(art) == int((din * dout).sum())
    assert (et == 1).sum() == int((dout * (dout - 1) // 2).sum())
    assert (et == 2).sum() == int((din * (din - 1) // 2).sum())
    # canonical order: articulations by (common hit, a, b)
    key = [(int(dst[a]), int(a), int(b)) for a, b in art]
    assert key == sorted(key)


def test_triplet_classifier_special_cases():
    H = 4
    rng = np.random.default_rng(3)
    e = rng.normal(0, 1, (6, H))
    pairs = np.array([[0, 1], [2, 1], [0, 3], [4, 5]], np.int32)
    tb = np.zeros(oracle.triplet_param_count(H), np.float32)
    per = H * 2 * H + H + H + 1
    assert tb.shape[0] == 2 * per
    for which in (0, 1):
        o = which * per
        W1 = tb[o:o + 2 * H * H].reshape(H, 2 * H)
        b1 = tb[o + 2 * H * H:o + 2 * H * H + H]
        W2 = tb[o + 2 * H * H + H:o + 2 * H * H + 2 * H]
        b2 = tb[o + 2 * H * H + 2 * H:o + per]
        # zero first layer: z = W2 relu(b1) + b2 for every triplet
        W1[:] = 0
        b1[:] = [0.5, -1.0, 2.0, 0.25]
        W2[:] = [1.0, 3.0, -0.5, 2.0]
        b2[:] = [-0.75]
        z = oracle.triplet_logits(pairs, e, tb, which)
        np.testing.assert_array_equal(z, np.full(4, 0.5 - 1.0 + 0.5 - 0.75))
        # first half only: z = sum relu(e_a) + b2 (triplets with the same a agree)
        W1[:] = 0
        W1[:, :H] = np.eye(H)
        b1[:] = 0
        W2[:] = 1
        b2[:] = 0
        z = oracle.triplet_logits(pairs, e, tb, which)
        np.testing.assert_allclose(z, np.maximum(e[pairs[:, 0]], 0).sum(1), rtol=1e-15)
        # second half only
        W1[:] = 0
        W1[:, H:] = np.eye(H)
        z = oracle.triplet_logits(pairs, e, tb, which)
        np.testing.assert_allclose(z, np.maximum(e[pairs[:, 1]], 0).sum(1), rtol=1e-15)
    # the two classifiers read their own weights
    tb[:] = 0
    tb[2 * H * H + 2 * H] = 1.5                     # articulation output bias
    tb[per + 2 * H * H + 2 * H] = -2.0              # elbow output bias
    assert np.all(oracle.triplet_logits(pairs, e, tb, 0) == 1.5)
    assert np.all(oracle.triplet_logits(pairs, e, tb, 1) == -2.0)


def _build(n, plane, edges, art_keep=None, elb_keep=None):
    edges = sorted(edges)
    src = np.array([a for a, _ in edges], np.int32)
    dst = np.array([b for _, b in edges], np.int32)
    keep = np.ones(len(edges), np.uint8)
    art, elb, et = oracle.triplets(n, src, dst, keep)
    idx = {e: q for q, e in enumerate(edges)}
    ak = np.ones(len(art), np.uint8) if art_keep is None else np.array(
        [art_keep((edges[a], edges[b])) for a, b in art], np.uint8)
    ek = np.ones(len(elb), np.uint8) if elb_keep is None else np.array(
        [elb_keep((edges[a], edges[b])) for a, b in elb], np.uint8)
    seg, tracks = oracle.build_tracks(n, src, dst, np.asarray(plane, np.int32), keep, art, ak, elb, ek)
    hits = oracle.track_hits(src, dst, seg, tracks)
    return idx, seg, tracks, sorted(tuple(h.tolist()) for h in hits)


def test_chain_is_one_track():
    idx, seg, tracks, hits = _build(5, [0, 1, 2, 3, 4], [(0, 1), (1, 2), (2, 3), (3, 4)])
    assert hits == [(0, 1, 2, 3, 4)]
    assert np.all(seg == 0) and tracks.tolist() == [[0, -1]]


def test_tracks_sharing_their_first_hits():
    """Hits 0 (plane 0) and 1 (plane 1) are shared; the tracks part at hit 1
    towards 2, 3 (planes 2, 3) and 4, 5 (planes 2, 3).  The left elbow at hit
    1 is rejected (its edges belong to different particles)."""
    plane = [0, 1, 2, 3, 2, 3]
    edges = [(0, 1), (1, 2), (2, 3), (1, 4), (4, 5)]
    idx, seg, tracks, hits = _build(6, plane, edges, elb_keep=lambda t: 0)
    assert hits == [(0, 1, 2, 3), (0, 1, 4, 5)]
    # the shared edge 0 -> 1 is its own segment, copied into both tracks
    assert seg[idx[(0, 1)]] == idx[(0, 1)]
    assert seg[idx[(1, 2)]] == seg[idx[(2, 3)]] != seg[idx[(1, 4)]] == seg[idx[(4, 5)]]
    assert len(tracks) == 2 and all(t[1] >= 0 for t in tracks.tolist())
    # with the elbow kept the two branches are one segment: both shared
    # articulations then make the same track (a clone, one per articulation)
    _, _, _, hits2 = _build(6, plane, edges)
    assert hits2 == [(0, 1, 2, 3, 4, 5)] * 2


def test_plane_skipping_edge_is_a_duplicate():
    """Hits 0..3 on planes 0..3 with edges 0->1, 1->2, 2->3 and the skip 0->2.
    The elbows (0->1, 0->2) and (0->2, 1->2) join the skip edge to the track
    and mark it a duplicate; without that, the articulations (0->2, 2->3) and
    (1->2, 2->3) would share 2->3 and split the track."""
    plane = [0, 1, 2, 3]
    edges = [(0, 1), (0, 2), (1, 2), (2, 3)]
    idx, seg, tracks, hits = _build(4, plane, edges)
    assert hits == [(0, 1, 2, 3)]
    assert len(tracks) == 1 and tracks[0, 1] == -1
    assert np.all(seg == 0)


def test_fake_bridge_with_rejected_triplets():
    """Tracks 0-1-2-3 and 4-5-6-7 (planes 0..3) and a kept fake edge 1 -> 6.
    Connected components of the kept hit graph give one component of 8 hits;
    with every triplet through the fake edge rejected, the edge graph gives
    the two tracks and the bridge as a two-hit candidate."""
    plane = [0, 1, 2, 3, 0, 1, 2, 3]
    edges = [(0, 1), (1, 2), (2, 3), (4, 5), (5, 6), (6, 7), (1, 6)]
    fake = (1, 6)
    reject = lambda t: 0 if fake in t else 1
    idx, seg, tracks, hits = _build(8, plane, edges, art_keep=reject, elb_keep=reject)
    assert hits == [(0, 1, 2, 3), (1, 6), (4, 5, 6, 7)]
    src = np.array([a for a, _ in sorted(edges)], np.int32)
    dst = np.array([b for _, b in sorted(edges)], np.int32)
    lab = oracle.components(8, src, dst, np.ones(len(edges), np.uint8))
    assert len(set(lab.tolist())) == 1


def test_track_list_metrics_equal_label_metrics_on_components():
    rng = np.random.default_rng(5)
    labels, pid, off = [], [], [0]
    for _ in range(4):
        n = int(rng.integers(30, 60))
        lab = rng.integers(0, n // 3, n)               # arbitrary labels
        labels.append(lab)
        pid.append(np.where(rng.random(n) < 0.1, -1, rng.integers(0, n // 4, n)))
        off.append(off[-1] + n)
    labels, pid = np.concatenate(labels), np.concatenate(pid)
    a = metrics.track_metrics(labels, pid, off)
    b = metrics.track_list_metrics(metrics.labels_to_tracks(labels, off), pid, off)
    for k in ("efficiency", "clone_rate", "fake_rate", "hit_efficiency", "hit_purity", "n_tracks", "n_pairs"):
        assert a[k] == pytest.approx(b[k], rel=1e-12), k


@pytest.mark.parametrize("which", [0, 1])
def test_triplet_classifier_gradient_against_finite_differences(which):
    """The numpy backward of the triplet classifiers against central
    differences of the C forward (independent code).  Inputs are dyadic, so
    every perturbed float32 parameter is exact, and every hidden unit's
    pre-activation stays on one side of zero (|W0 x| <= 1/2 < |b0|): the
    logits are then linear in each parameter and the differences exact up to
    float64 rounding."""
    H = 4
    rng = np.random.default_rng(11 + which)
    q = lambda a: np.round(a * 1024) / 1024
    e = q(rng.uniform(-1, 1, (7, H)))
    pairs = np.array([[0, 1], [2, 1], [0, 3], [4, 5], [6, 2], [5, 0]], np.int32)
    per = 2 * H * H + 2 * H + 1
    tb = np.zeros(2 * per, np.float32)
    for w in (0, 1):
        o = w * per
        tb[o:o + 2 * H * H] = q(rng.uniform(-1, 1, 2 * H * H) / 16)
        tb[o + 2 * H * H:o + 2 * H * H + H] = [1.0, -1.0, 1.5, -0.75]
        tb[o + 2 * H * H + H:o + per] = q(rng.uniform(-1, 1, H + 1))
    dz = rng.normal(0, 1, len(pairs))
    g = oracle.triplet_classifier_grad(pairs, e, tb, which, dz)
    assert g.shape == (per,)
    h = 2.0 ** -6
    f = lambda b: float(dz @ oracle.triplet_logits(pairs, e, b, which))
    for k in range(per):
        bp, bm = tb.copy(), tb.copy()
        bp[which * per + k] += h
        bm[which * per + k] -= h
        assert bp[which * per + k] - tb[which * per + k] == h      # exact in float32
        fd = (f(bp) - f(bm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-12 * max(1.0, abs(fd)), (k, fd, g[k])
    # the other classifier's parameters do not move these logits
    other = tb.copy()
    other[(1 - which) * per:(2 - which) * per] += np.float32(0.5)
    assert f(other) == f(tb)


def test_track_hit_lists_equal_the_oracle_track_hits():
    """metrics.track_hit_lists (host code that scores the GPU's tracks) gives
    the oracle's hit lists on random graphs with random triplet decisions."""
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        plane, src, dst = _random_graph(rng, n=30, m=60)
        keep = (rng.random(len(src)) < 0.7).astype(np.uint8)
        art, elb, et = oracle.triplets(30, src, dst, keep)
        ak = (rng.random(len(art)) < 0.6).astype(np.uint8)
        ek = (rng.random(len(elb)) < 0.3).astype(np.uint8)
        seg, tracks = oracle.build_tracks(30, src, dst, plane, keep, art, ak, elb, ek)
        want = oracle.track_hits(src, dst, seg, tracks)
        got = metrics.track_hit_lists(src, dst, seg, tracks)
        assert len(got) == len(want)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
