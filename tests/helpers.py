"""Shared test helpers: structured parameter blobs and small graphs.

Only the tests import this module.  It builds inputs; it holds none of the
track-finding arithmetic.
"""
import numpy as np

from paper_2407_12119_amd import synth


def zero_blob(H, iters, Ce=128, D=4, norm=None):
    blob = np.zeros(synth.param_count(H, iters, Ce, D), np.float32)
    if norm is None:
        norm = [0, 0, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1]
    blob[:12] = np.asarray(norm, np.float32)
    return blob, synth.param_views(blob, H, iters, Ce, D)


def random_graph(n, n_edges, rng, planes=None):
    """Distinct directed edges src -> dst with src != dst, sorted by (src, dst)."""
    pairs = set()
    while len(pairs) < n_edges:
        a, b = (int(v) for v in rng.integers(0, n, 2))
        if a != b:
            pairs.add((a, b))
    e = np.array(sorted(pairs), np.int32).reshape(-1, 2)
    return e[:, 0].copy(), e[:, 1].copy()
