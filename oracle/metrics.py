"""Track-finding metrics, written out with plain loops over hits.

TEST INFRASTRUCTURE ONLY (part of the oracle): the tests, the smoke check and
the benchmark's CPU baseline leg may use it; the product path never does.

Definitions (Physics Performance section and its metrics table; reconstructible
particles as in the detector section):
  * a track (candidate) is a connected component of at least 3 hits;
  * a particle is reconstructible if it left at least 3 hits in the event;
  * a track matches a particle when at least 70% of the track's hits carry
    that particle's id (noise hits carry none); at most one particle can
    reach 70%, and any matched particle has at least 3 hits;
  * efficiency = matched particles / reconstructible particles;
  * clone rate = (matching pairs - matched particles) / matching pairs;
  * fake rate = unmatched tracks / tracks;
  * hit efficiency and hit purity are means over matching pairs of
    (track hits of the particle) / (particle hits) and / (track hits).
Counts are pooled over all events.  A ratio whose denominator is 0 is reported
as 0 and its name is listed under "undefined".
"""
from __future__ import annotations

from fractions import Fraction


def track_metrics(labels_per_event, pid_per_event, min_track_hits: int = 3, match_frac=Fraction(7, 10),
                  min_particle_hits: int = 3):
    n_particles = n_tracks = n_fake = n_pairs = n_matched_particles = 0
    sum_hit_eff = Fraction(0)
    sum_purity = Fraction(0)
    for labels, pid in zip(labels_per_event, pid_per_event):
        labels = [int(v) for v in labels]
        pid = [int(v) for v in pid]
        assert len(labels) == len(pid)
        particle_hits = {}
        for p in pid:
            if p != -1:
                particle_hits[p] = particle_hits.get(p, 0) + 1
        n_particles += sum(1 for c in particle_hits.values() if c >= min_particle_hits)
        members = {}
        for i, l in enumerate(labels):
            members.setdefault(l, []).append(i)
        matched = set()
        for l, hits in members.items():
            if len(hits) < min_track_hits:
                continue
            n_tracks += 1
            counts = {}
            for i in hits:
                if pid[i] != -1:
                    counts[pid[i]] = counts.get(pid[i], 0) + 1
            best = None
            for p, c in counts.items():
                if Fraction(c, len(hits)) >= match_frac:
                    best = p
            if best is None:
                n_fake += 1
                continue
            n_pairs += 1
            matched.add(best)
            sum_hit_eff += Fraction(counts[best], particle_hits[best])
            sum_purity += Fraction(counts[best], len(hits))
        n_matched_particles += len(matched)
    undefined = []

    def ratio(num, den, name):
        if den == 0:
            undefined.append(name)
            return 0.0
        return float(Fraction(num) / den)

    return {
        "efficiency": ratio(n_matched_particles, n_particles, "efficiency"),
        "clone_rate": ratio(n_pairs - n_matched_particles, n_pairs, "clone_rate"),
        "fake_rate": ratio(n_fake, n_tracks, "fake_rate"),
        "hit_efficiency": ratio(sum_hit_eff, n_pairs, "hit_efficiency"),
        "hit_purity": ratio(sum_purity, n_pairs, "hit_purity"),
        "n_particles": n_particles, "n_tracks": n_tracks, "n_matched_particles": n_matched_particles,
        "n_pairs": n_pairs, "n_fake": n_fake, "undefined": undefined,
    }
