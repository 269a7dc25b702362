"""Track-finding metrics of a labelled batch (Physics Performance section,
metrics table), vectorised over the whole batch on the host.

A track is a connected component of >= 3 hits; a particle with >= 3 hits in
its event is reconstructible; a track matches a particle when >= 70% of its
hits carry that particle's id.  Efficiency, clone rate and fake rate are pooled
over all events; hit efficiency and hit purity are means over the matching
(track, particle) pairs.  A ratio with a zero denominator is 0 and is listed
under "undefined".

Inputs are the batch-wide arrays the pipeline returns: `labels` (event-local
component label per hit), `pid` (particle id per hit, -1 for noise, ids local
to an event) and `event_offsets` [B+1].
"""
from __future__ import annotations

import numpy as np

MIN_TRACK_HITS = 3
MIN_PARTICLE_HITS = 3
MATCH_NUM, MATCH_DEN = 7, 10      # 70%, compared in integers: 10 * count >= 7 * size


def track_metrics(labels, pid, event_offsets) -> dict:
    labels = np.asarray(labels, np.int64)
    pid = np.asarray(pid, np.int64)
    off = np.asarray(event_offsets, np.int64)
    n = labels.shape[0]
    ev = np.repeat(np.arange(off.shape[0] - 1, dtype=np.int64), np.diff(off))
    assert ev.shape[0] == n == pid.shape[0]

    # tracks: (event, label) groups
    _, track, track_size = np.unique(np.stack([ev, labels], 1), axis=0, return_inverse=True,
                                     return_counts=True)
    track = track.reshape(-1)
    is_track = track_size >= MIN_TRACK_HITS
    n_tracks = int(is_track.sum())

    # particles: (event, pid) groups over signal hits
    sig = pid >= 0
    _, part, part_size = np.unique(np.stack([ev[sig], pid[sig]], 1), axis=0, return_inverse=True,
                                   return_counts=True)
    part = part.reshape(-1)
    n_particles = int((part_size >= MIN_PARTICLE_HITS).sum())

    # (track, particle) hit counts
    t_sig = track[sig]
    pairs, pair_count = np.unique(np.stack([t_sig, part], 1), axis=0, return_counts=True)
    pt, pp = pairs[:, 0], pairs[:, 1]
    match = is_track[pt] & (MATCH_DEN * pair_count >= MATCH_NUM * track_size[pt])
    pt, pp, pc = pt[match], pp[match], pair_count[match]
    n_pairs = int(pt.shape[0])
    n_matched = int(np.unique(pp).shape[0])
    n_fake = n_tracks - n_pairs
    undefined = []

    def ratio(num, den, name):
        if den == 0:
            undefined.append(name)
            return 0.0
        return float(num) / float(den)

    return {
        "efficiency": ratio(n_matched, n_particles, "efficiency"),
        "clone_rate": ratio(n_pairs - n_matched, n_pairs, "clone_rate"),
        "fake_rate": ratio(n_fake, n_tracks, "fake_rate"),
        "hit_efficiency": ratio(np.sum(pc / part_size[pp]), n_pairs, "hit_efficiency"),
        "hit_purity": ratio(np.sum(pc / track_size[pt]), n_pairs, "hit_purity"),
        "n_particles": n_particles, "n_tracks": n_tracks, "n_matched_particles": n_matched,
        "n_pairs": n_pairs, "n_fake": n_fake, "undefined": undefined,
    }


def edge_keys(off, src, dst) -> np.ndarray:
    """One int64 key per edge: (event, event-local src, event-local dst)."""
    ev = np.repeat(np.arange(len(off) - 1, dtype=np.int64), np.diff(np.asarray(off, np.int64)))
    return (ev << 42) | (np.asarray(src, np.int64) << 21) | np.asarray(dst, np.int64)


def edge_agreement(a_off, a_src, a_dst, a_keep, b_off, b_src, b_dst, b_keep) -> dict:
    """Agreement of the keep decisions of two edge sets of one batch, over
    the union of their edges (an edge absent from a set counts as rejected
    there), and the Jaccard overlap of the two edge sets."""
    ka, kb = edge_keys(a_off, a_src, a_dst), edge_keys(b_off, b_src, b_dst)
    u = np.union1d(ka, kb)
    da = np.zeros(u.shape[0], bool)
    db = np.zeros(u.shape[0], bool)
    da[np.searchsorted(u, ka)] = np.asarray(a_keep, bool)
    db[np.searchsorted(u, kb)] = np.asarray(b_keep, bool)
    inter = np.intersect1d(ka, kb).shape[0]
    return {"decision_agreement": float((da == db).mean()) if u.shape[0] else 1.0,
            "jaccard": float(inter / u.shape[0]) if u.shape[0] else 1.0,
            "n_union": int(u.shape[0])}


def track_list_metrics(tracks, pid, event_offsets) -> dict:
    """The same metrics for tracks given as hit lists, which may share hits
    (tracks built from the purified edge graph, Sec. 5.4).  `tracks[b]` is the
    list of event b's tracks, each an array of event-local hit indices
    without repeats; a track needs >= 3 hits.  Matching, efficiency, clone
    rate, fake rate, hit efficiency and hit purity as in track_metrics."""
    pid = np.asarray(pid, np.int64)
    off = np.asarray(event_offsets, np.int64)
    n_particles = n_tracks = n_pairs = n_matched = 0
    he = hp = 0.0
    undefined = []
    for b in range(off.shape[0] - 1):
        p = pid[off[b]:off[b + 1]]
        sig = p[p >= 0]
        ids, sizes = np.unique(sig, return_counts=True)
        size_of = dict(zip(ids.tolist(), sizes.tolist()))
        n_particles += int((sizes >= MIN_PARTICLE_HITS).sum())
        matched = set()
        for t in tracks[b]:
            t = np.asarray(t, np.int64)
            if t.shape[0] < MIN_TRACK_HITS:
                continue
            n_tracks += 1
            tp = p[t]
            tp = tp[tp >= 0]
            if tp.shape[0] == 0:
                continue
            cand, cnt = np.unique(tp, return_counts=True)
            for q, c in zip(cand.tolist(), cnt.tolist()):
                if MATCH_DEN * c >= MATCH_NUM * t.shape[0]:
                    n_pairs += 1
                    matched.add(q)
                    he += c / size_of[q]
                    hp += c / t.shape[0]
        n_matched += len(matched)

    def ratio(num, den, name):
        if den == 0:
            undefined.append(name)
            return 0.0
        return float(num) / float(den)

    return {
        "efficiency": ratio(n_matched, n_particles, "efficiency"),
        "clone_rate": ratio(n_pairs - n_matched, n_pairs, "clone_rate"),
        "fake_rate": ratio(n_tracks - n_pairs, n_tracks, "fake_rate"),
        "hit_efficiency": ratio(he, n_pairs, "hit_efficiency"),
        "hit_purity": ratio(hp, n_pairs, "hit_purity"),
        "n_particles": n_particles, "n_tracks": n_tracks, "n_matched_particles": n_matched,
        "n_pairs": n_pairs, "n_fake": n_tracks - n_pairs, "undefined": undefined,
    }


def track_hit_lists(src, dst, edge_seg, tracks):
    """One event's tracks from the purified edge graph (Sec. 5.4) as hit
    lists: a track is one or two segments (`tracks` [T x 2] of segment
    labels, the second -1 for one segment), a segment the kept edges with
    that label (`edge_seg`, -1 for other edges), and a track's hits the ends
    of its edges, ascending, without repeats (step 4, edges replaced by
    hits)."""
    src, dst = np.asarray(src, np.int64), np.asarray(dst, np.int64)
    seg = np.asarray(edge_seg, np.int64)
    tracks = np.asarray(tracks, np.int64).reshape(-1, 2)
    ends = {}
    kept = np.nonzero(seg >= 0)[0]
    if kept.shape[0]:
        order = kept[np.argsort(seg[kept], kind="stable")]
        labs, first = np.unique(seg[order], return_index=True)
        for lab, grp in zip(labs.tolist(), np.split(order, first[1:])):
            ends[lab] = np.unique(np.concatenate([src[grp], dst[grp]]))
    out = []
    for a, b in tracks.tolist():
        h = ends.get(a, np.zeros(0, np.int64))
        if b >= 0:
            h = np.union1d(h, ends.get(b, np.zeros(0, np.int64)))
        out.append(h.astype(np.int32))
    return out


def labels_to_tracks(labels, event_offsets):
    """Connected-component labels -> per-event lists of hit arrays (one per component)."""
    labels = np.asarray(labels, np.int64)
    off = np.asarray(event_offsets, np.int64)
    out = []
    for b in range(off.shape[0] - 1):
        lab = labels[off[b]:off[b + 1]]
        order = np.argsort(lab, kind="stable")
        _, first = np.unique(lab[order], return_index=True)
        out.append(np.split(order, first[1:]) if lab.shape[0] else [])
    return out
