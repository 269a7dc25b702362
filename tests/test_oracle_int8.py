"""Pins of the oracle's INT8 embedding (Sec. 7.4: the embedding MLP run with
INT8 operands under static per-tensor scales calibrated on a set of events).

* A network whose every operand sits exactly on its INT8 grid: the INT8
  result must equal the float64 embedding exactly, and a hand computation
  from the integer codes.  Scales are powers of two set by the calibration
  maxima, so a swapped scale, a missing descale, a transposed weight or a
  misplaced ReLU changes the result.
* Ties of the code rounding go to the even integer; values beyond the
  calibrated range clamp to +-127.
* On the seeded init the INT8 embedding stays within the error bound of
  per-tensor quantisation (half a step of each operand, propagated through
  the two layers).
"""
import numpy as np
import pytest

import oracle
from paper_2407_12119_amd import synth

from helpers import zero_blob

CE, D = 128, 4


def _grid_network():
    blob, v = zero_blob(4, 0)
    W1, b1 = v["emb0"]
    W2, b2 = v["emb1"]
    W3, b3 = v["emb2"]
    k = np.zeros(CE)
    k[0], k[1], k[2] = 127, 2, 3            # first hidden layer = relu(b1) = k / 16 (W1 = 0)
    b1[:] = k / 16
    m = np.zeros((CE, CE))
    m[0, 1], m[0, 2] = 2, 41                # 2*2 + 3*41 = 127: the largest second-layer output
    m[1, 1], m[1, 2] = -5, 7                # 11
    m[2, 1], m[2, 2] = 10, -10              # -10 -> ReLU -> 0
    m[3, 1], m[3, 2] = 1, 1                 # 5
    m[5, 7] = 127                           # sets max |W2| = 127 / 32; k[7] = 0
    W2[:] = m / 32
    p = np.zeros((D, CE))
    p[0, 0], p[0, 1] = 3, -127
    p[1, 3], p[2, 0], p[3, 1], p[3, 3] = 50, -7, 1, 2
    W3[:] = p / 64
    b3[:] = [0.25, -1.5, 3.0, 0.0]
    # second-layer outputs h2 = (k m^T) / 512, their codes under s_x3 = 1/512
    h2_codes = np.maximum(k @ m.T, 0)
    expect = (p @ h2_codes) / 512 / 64 + b3
    return blob, h2_codes, expect


def _hits(n=7, seed=0):
    rng = np.random.default_rng(seed)
    r = rng.uniform(6, 40, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    z = rng.uniform(-290, 750, n)
    return (r * np.cos(phi)).astype(np.float32), (r * np.sin(phi)).astype(np.float32), z.astype(np.float32)


def test_grid_network_is_exact():
    blob, codes, expect = _grid_network()
    x, y, z = _hits()
    ev = synth.Event(x, y, z, np.zeros(len(x), np.int32), np.zeros(len(x), np.int64), np.full(len(x), -1, np.int32))
    amax = oracle.embed_amax([ev], blob)
    assert amax[0] == 127 / 16 and amax[1] == 127 / 512
    sc = oracle.int8_scales(amax, blob)
    np.testing.assert_array_equal(sc, np.float32([1 / 16, 1 / 32, 1 / 512, 1 / 64]))
    assert codes.max() == 127
    e8 = oracle.embed_int8(x, y, z, blob, sc)
    e64 = oracle.embed(x, y, z, blob)
    for i in range(len(x)):
        np.testing.assert_array_equal(e8[i], expect)
        np.testing.assert_array_equal(e64[i], expect)


def test_code_ties_round_to_even_and_clamp():
    blob, _, _ = _grid_network()
    v = synth.param_views(blob, 4, 0)
    b1 = v["emb0"][1]
    W2 = v["emb1"][0]
    b1[:] = 0
    b1[0], b1[1] = 2.5 / 16, 3.5 / 16        # ties: codes 2 and 4
    b1[2] = 300 / 16                          # beyond the scale's range: code 127
    W2[:] = 0
    W2[0, 0], W2[0, 1], W2[0, 2] = 1 / 32, 1 / 32, 1 / 32
    W2[5, 7] = 127 / 32
    x, y, z = _hits(3)
    sc = np.float32([1 / 16, 1 / 32, 1 / 512, 1 / 64])
    e8 = oracle.embed_int8(x, y, z, blob, sc)
    W3 = v["emb2"][0]
    b3 = v["emb2"][1]
    h2 = (2 + 4 + 127) / 512                  # codes 2 + 4 + 127 times s_x2 s_w2 = 1/512
    q3 = min(round(h2 * 512), 127)            # the layer-3 code of h2 under s_x3 = 1/512 (127)
    expect = (np.rint(W3[:, 0] * 64) * q3) / 512 / 64 + b3.astype(np.float64)
    np.testing.assert_array_equal(e8[0], expect)


def test_seeded_init_within_the_quantisation_bound():
    """|e_int8 - e_64| per output <= the propagated half-step bound:
    layer 2: |dz2_c| <= sum_j |W2_cj| s_x2 / 2 + sum_j |h1_j| s_w2 / 2 + K s_x2 s_w2 / 4,
    ReLU is 1-Lipschitz, layer 3 likewise with |W3| and the perturbed h2."""
    wl = synth.WORKLOADS["batch256"]
    blob = synth.init_params(wl)
    evs = synth.make_events(wl, 3, first=4)
    amax = oracle.embed_amax(evs, blob)
    sc = oracle.int8_scales(amax, blob).astype(np.float64)
    v = synth.param_views(blob, wl.hidden, wl.iters)
    W1, b1 = (a.astype(np.float64) for a in v["emb0"])
    W2, b2 = (a.astype(np.float64) for a in v["emb1"])
    W3 = v["emb2"][0].astype(np.float64)
    norm = blob[:12].astype(np.float64)
    for ev in evs:
        e8 = oracle.embed_int8(ev.x, ev.y, ev.z, blob, sc.astype(np.float32))
        e64 = oracle.embed(ev.x, ev.y, ev.z, blob)
        X, Y, Z = (a.astype(np.float64) for a in (ev.x, ev.y, ev.z))
        u = np.stack([(np.hypot(X, Y) - norm[0]) / norm[3], (np.arctan2(Y, X) - norm[1]) / norm[4],
                      (Z - norm[2]) / norm[5]], 1)
        h1 = np.maximum(u @ W1.T + b1, 0)
        h2 = np.maximum(h1 @ W2.T + b2, 0)
        d2 = (np.abs(W2).sum(1) * sc[0] / 2 + np.abs(h1).sum(1)[:, None] * sc[1] / 2
              + CE * sc[0] * sc[1] / 4)
        bound = (np.abs(W3) @ (d2.T)).T + (np.abs(W3).sum(1) * sc[2] / 2 + (np.abs(h2) + d2).sum(1)[:, None]
                                            * sc[3] / 2 + CE * sc[2] * sc[3] / 4)
        err = np.abs(e8 - e64)
        assert np.all(err <= bound * (1 + 1e-9) + 1e-12), (err / bound).max()
        assert err.max() > 0                    # the operands really are quantised
        print(f"  {ev.n} hits: max |de| {err.max():.3g}, max of err / bound {(err / bound).max():.3f}")


def test_planted_mistakes_fail_a_pin():
    """The grid network separates the scales of the two layers: using the
    second layer's input scale for the third layer (a plausible slip) changes
    the result."""
    blob, _, expect = _grid_network()
    x, y, z = _hits(2)
    swapped = np.float32([1 / 16, 1 / 32, 1 / 16, 1 / 64])
    e8 = oracle.embed_int8(x, y, z, blob, swapped)
    assert not np.array_equal(e8[0], expect)
