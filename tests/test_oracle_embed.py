"""Pins of the oracle's feature normalisation and embedding MLP (Sec. 5.1).

Expected values are derived by hand from the definitions (r = sqrt(x^2+y^2),
phi = atan2(y, x), ReLU between layers, linear output), never by running the
oracle's own code path.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import zero_blob
from paper_2407_12119_amd import synth

HITS = np.array([[3.0, 4.0, 10.0],     # r = 5, phi = atan2(4, 3)
                 [0.0, -5.0, -2.0],    # r = 5, phi = -pi/2
                 [-1.0, 0.0, 0.0]],    # r = 1, phi = pi
                np.float32)


def _emb(blob):
    return oracle.embed(HITS[:, 0], HITS[:, 1], HITS[:, 2], blob)


def test_handcrafted_relu_network():
    blob, v = zero_blob(8, 0)
    W1, b1 = v["emb0"]; W2, b2 = v["emb1"]; W3, b3 = v["emb2"]
    W1[0, 0] = 1; b1[0] = -4          # relu(r - 4)
    W1[1, 1] = 1                      # relu(phi)
    W1[2, 2] = 1                      # relu(z)
    W2[0, 0] = 1                      # relu(h0)
    W2[1, 1] = -1; b2[1] = 1          # relu(1 - h1)
    W2[2, 2] = 0.5                    # relu(h2 / 2)
    W3[0, 0] = 1; W3[0, 1] = 1        # out0 = g0 + g1
    W3[1, 2] = -1; b3[1] = 3          # out1 = 3 - g2
    W3[2, 1] = 2                      # out2 = 2 g1
    b3[3] = -1                        # out3 = -1
    phiA = math.atan2(4.0, 3.0)       # 0.9272952180016122
    exp = np.array([
        [1 + (1 - phiA), 3 - 5.0, 2 * (1 - phiA), -1],
        [1 + 1, 3 - 0.0, 2 * 1, -1],          # phi = -pi/2 -> relu 0; z = -2 -> relu 0
        [0 + 0, 3 - 0.0, 0, -1],              # r - 4 < 0; 1 - pi < 0
    ])
    np.testing.assert_allclose(_emb(blob), exp, rtol=0, atol=1e-15)


def test_normalisation_constants():
    """u = (f - mu) / sigma per feature; with an identity network the output is u."""
    norm = [1, 0.5, 2, 2, 4, 0.5, 0, 0, 0, 1, 1, 1]
    blob, v = zero_blob(8, 0, norm=norm)
    W1, b1 = v["emb0"]; W2, b2 = v["emb1"]; W3, b3 = v["emb2"]
    for c in range(3):
        W1[c, c] = 1; b1[c] = 100      # keep every ReLU in its linear part
        W2[c, c] = 1
        W3[c, c] = 1; b3[c] = -100
    phiA = math.atan2(4.0, 3.0)
    exp = np.array([[(5 - 1) / 2, (phiA - 0.5) / 4, (10 - 2) / 0.5, 0],
                    [(5 - 1) / 2, (-math.pi / 2 - 0.5) / 4, (-2 - 2) / 0.5, 0],
                    [(1 - 1) / 2, (math.pi - 0.5) / 4, (0 - 2) / 0.5, 0]])
    np.testing.assert_allclose(_emb(blob), exp, rtol=0, atol=1e-12)


def test_linear_regime_equals_collapsed_affine_map():
    """With every ReLU active the MLP is the affine map W3 W2 W1 u + (W3 W2 b1 + W3 b2 + b3)."""
    rng = np.random.default_rng(5)
    blob, v = zero_blob(8, 0)
    W1, b1 = v["emb0"]; W2, b2 = v["emb1"]; W3, b3 = v["emb2"]
    W1[:] = rng.uniform(-1, 1, W1.shape); b1[:] = 50
    W2[:] = rng.uniform(0, 1, W2.shape) / 128; b2[:] = rng.uniform(0, 1, 128)
    W3[:] = rng.uniform(-1, 1, W3.shape); b3[:] = rng.uniform(-1, 1, 4)
    f = np.array([[5, math.atan2(4, 3), 10], [5, -math.pi / 2, -2], [1, math.pi, 0]])
    A = W3.astype(np.float64) @ W2.astype(np.float64) @ W1.astype(np.float64)
    c = W3.astype(np.float64) @ (W2.astype(np.float64) @ b1 + b2) + b3
    exp = f @ A.T + c
    np.testing.assert_allclose(_emb(blob), exp, rtol=1e-12, atol=1e-12)


def test_zero_weights_give_output_bias():
    blob, v = zero_blob(8, 0)
    v["emb2"][1][:] = [0.25, -1.5, 3.0, 7.0]
    np.testing.assert_array_equal(_emb(blob), np.tile([0.25, -1.5, 3.0, 7.0], (3, 1)))


def test_embedding_is_per_hit():
    """Each hit's embedding depends on that hit alone (order and batch do not matter)."""
    wl = synth.WORKLOADS["single_event"]
    ev = synth.make_events(wl)[0]
    blob = synth.init_params(wl)
    full = oracle.embed(ev.x, ev.y, ev.z, blob)
    perm = np.random.default_rng(0).permutation(ev.n)
    part = oracle.embed(ev.x[perm], ev.y[perm], ev.z[perm], blob)
    np.testing.assert_array_equal(full[perm], part)
