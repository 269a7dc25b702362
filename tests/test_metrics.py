"""Track-finding metrics (Physics Performance section, metrics table): the
oracle's loop version pinned on constructed cases worked out by hand from the
table's definitions, and the vectorised version in the package against it."""
import numpy as np
import pytest

import oracle
from oracle.metrics import track_metrics as ref_metrics
from paper_2407_12119_amd import metrics, synth


def _both(labels_list, pid_list):
    off = np.concatenate([[0], np.cumsum([len(l) for l in labels_list])]).astype(np.int32)
    lab = np.concatenate(labels_list) if labels_list else np.zeros(0, np.int64)
    pid = np.concatenate(pid_list) if pid_list else np.zeros(0, np.int64)
    return ref_metrics(labels_list, pid_list), metrics.track_metrics(lab, pid, off)


def _same(a, b):
    for k in a:
        if k == "undefined":
            assert sorted(a[k]) == sorted(b[k])
        else:
            assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-15), k


def test_perfect_classifier_finds_every_reconstructible_particle():
    # particles 0 (4 hits), 1 (3 hits), 2 (2 hits: not reconstructible), noise
    pid = np.array([0, 0, 0, 0, 1, 1, 1, 2, 2, -1])
    labels = np.array([0, 0, 0, 0, 4, 4, 4, 7, 7, 9])
    a, b = _both([labels], [pid])
    _same(a, b)
    assert a["n_particles"] == 2 and a["n_tracks"] == 2
    assert a["efficiency"] == 1.0 and a["clone_rate"] == 0.0 and a["fake_rate"] == 0.0
    assert a["hit_efficiency"] == 1.0 and a["hit_purity"] == 1.0 and a["undefined"] == []


def test_all_reject_gives_no_tracks():
    pid = np.array([0, 0, 0, 1, 1, 1, -1])
    a, b = _both([np.arange(7)], [pid])
    _same(a, b)
    assert a["n_tracks"] == 0 and a["efficiency"] == 0.0 and a["fake_rate"] == 0.0
    assert set(a["undefined"]) == {"fake_rate", "clone_rate", "hit_efficiency", "hit_purity"}


def test_merged_tracks_and_the_seventy_percent_rule():
    # event 1: one component with 3 hits of A and 3 of B -> 50% each: a fake track
    # event 2: 7 hits of A and 3 of B -> matched to A, purity 0.7; B (3 hits) unmatched
    # event 3: 2 hits of A + 1 noise -> 2/3 < 70%: fake
    e1 = (np.zeros(6, int), np.array([0, 0, 0, 1, 1, 1]))
    e2 = (np.zeros(10, int), np.array([5] * 7 + [6] * 3))
    e3 = (np.array([0, 0, 0, 3, 4]), np.array([2, 2, -1, 2, 2]))
    a, b = _both([e1[0], e2[0], e3[0]], [e1[1], e2[1], e3[1]])
    _same(a, b)
    # particles: e1 A, B; e2 A(7), B(3); e3 A has 4 hits -> 5 reconstructible
    assert a["n_particles"] == 5 and a["n_tracks"] == 3 and a["n_fake"] == 2
    assert a["efficiency"] == pytest.approx(1 / 5)
    assert a["hit_purity"] == pytest.approx(0.7) and a["hit_efficiency"] == 1.0


def test_split_particle_is_a_clone():
    # one particle of 8 hits split into two tracks of 4, plus a 3-hit track of 5 noise-free hits of another
    pid = np.array([0] * 8 + [1] * 5)
    labels = np.array([0] * 4 + [4] * 4 + [8, 8, 8, 11, 12])
    a, b = _both([labels], [pid])
    _same(a, b)
    assert a["n_pairs"] == 3 and a["n_matched_particles"] == 2
    assert a["clone_rate"] == pytest.approx(1 / 3)
    assert a["hit_efficiency"] == pytest.approx((0.5 + 0.5 + 3 / 5) / 3)
    assert a["efficiency"] == 1.0


def test_noise_on_a_track_lowers_purity_only():
    pid = np.array([3] * 7 + [-1] * 3)
    a, b = _both([np.zeros(10, int)], [pid])
    _same(a, b)
    assert a["efficiency"] == 1.0 and a["hit_purity"] == pytest.approx(0.7) and a["hit_efficiency"] == 1.0


def test_empty_batch_and_empty_events():
    a, b = _both([np.zeros(0, int), np.zeros(0, int)], [np.zeros(0, int), np.zeros(0, int)])
    _same(a, b)
    assert a["n_particles"] == 0 and "efficiency" in a["undefined"]


def test_vectorised_metrics_equal_loop_metrics_on_oracle_components():
    rng = np.random.default_rng(11)
    events = synth.make_events(synth.WORKLOADS["batch256"], n_events=6)
    labs, pids = [], []
    for ev in events:
        n = ev.n
        if n < 2:
            labs.append(np.arange(n)); pids.append(ev.pid)
            continue
        # truth edges, a random fraction dropped, random fake edges added
        src = np.nonzero(ev.next_hit >= 0)[0].astype(np.int32)
        dst = ev.next_hit[src].astype(np.int32)
        keep = rng.random(src.shape[0]) < 0.9
        fs = rng.integers(0, n, n // 20).astype(np.int32)
        fd = rng.integers(0, n, n // 20).astype(np.int32)
        s = np.concatenate([src, fs]); d = np.concatenate([dst, fd])
        k = np.concatenate([keep, np.ones(fs.shape[0], bool)]).astype(np.uint8)
        labs.append(oracle.components(n, s, d, k))
        pids.append(ev.pid)
    a, b = _both(labs, pids)
    _same(a, b)
    assert 0.3 < a["efficiency"] <= 1.0 and a["n_tracks"] > 50


def test_edge_agreement_over_the_union():
    off = np.array([0, 3, 4])
    r = metrics.edge_agreement(off, [0, 0, 1, 2], [1, 2, 2, 0], [1, 0, 1, 1],
                               np.array([0, 2, 4]), [0, 1, 2, 1], [1, 2, 0, 0], [1, 1, 1, 0])
    # union: ev0 (0,1) (0,2) (1,2); ev1 (2,0) (1,0) -> 5 keys; decisions differ only on (0,2)? a rejects it,
    # b lacks it (rejected): equal.  (1,0) in ev1: b keeps? no (0).  a lacks it: equal.  all agree
    assert r["n_union"] == 5 and r["decision_agreement"] == 1.0 and r["jaccard"] == pytest.approx(3 / 5)
    r2 = metrics.edge_agreement(off, [0, 0, 1, 2], [1, 2, 2, 0], [1, 1, 1, 1],
                                np.array([0, 2, 4]), [0, 1, 2, 1], [1, 2, 0, 0], [1, 1, 1, 1])
    assert r2["decision_agreement"] == pytest.approx(3 / 5)
