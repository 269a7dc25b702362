"""Pins of the oracle's training form: weighted binary cross-entropy and the
reverse-mode gradient of the GNN (message passing, MLPs, encoders).

The gradient is checked against central finite differences of the oracle's
float64 forward pass, which shares no code with the backward pass.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import random_graph
from paper_2407_12119_amd import synth


def test_bce_closed_form_values():
    # z = 0: softplus(0) = ln 2 for both labels; dL/dz = w (1/2 - y) / E
    L, dz = oracle.bce(np.zeros(2), np.array([1, 0]), pos_weight=3.0)
    assert L == pytest.approx((3 * math.log(2) + math.log(2)) / 2, rel=1e-15)
    np.testing.assert_allclose(dz, [3 * (0.5 - 1) / 2, (0.5 - 0) / 2], rtol=1e-15)
    # large |z|: softplus(z) - y z -> 0 when the sign agrees with y
    L, dz = oracle.bce(np.array([40.0, -40.0]), np.array([1, 0]), pos_weight=2.0)
    assert L < 1e-16 and np.all(np.abs(dz) < 1e-16)
    L, _ = oracle.bce(np.zeros(0), np.zeros(0, np.uint8), 1.0)
    assert L == 0.0


def test_bce_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    z = rng.normal(0, 2, 50)
    yv = (rng.random(50) < 0.3).astype(np.uint8)
    _, dz = oracle.bce(z, yv, 2.5)
    h = 1e-6
    for q in range(0, 50, 7):
        zp, zm = z.copy(), z.copy()
        zp[q] += h; zm[q] -= h
        fd = (oracle.bce(zp, yv, 2.5)[0] - oracle.bce(zm, yv, 2.5)[0]) / (2 * h)
        assert fd == pytest.approx(dz[q], rel=1e-6, abs=1e-10)


@pytest.mark.parametrize("H,iters", [(4, 2), (8, 1)])
def test_gnn_gradient_matches_finite_differences(H, iters):
    rng = np.random.default_rng(H * 10 + iters)
    n = 9
    src, dst = random_graph(n, 20, rng)
    x, y, z = (rng.uniform(-20, 20, n).astype(np.float32) for _ in range(3))
    wl = synth.dataclasses.replace(synth.WORKLOADS["single_event"], hidden=H, iters=iters)
    blob = synth.init_params(wl)
    # wider weights than the default init so that no hidden layer is dead
    g0 = 12 + sum(o * i + o for _, (o, i) in synth.param_layout(H, iters)[:3])
    blob[g0:] = rng.uniform(-1, 1, blob.shape[0] - g0).astype(np.float32)
    dlogit = rng.normal(0, 1, src.shape[0])
    grad = oracle.gnn_backward(x, y, z, src, dst, blob, H, iters, dlogit)
    assert np.all(grad[:g0] == 0)

    def f(b):
        return float(dlogit @ oracle.gnn_forward(x, y, z, src, dst, b, H, iters))

    fd = np.zeros_like(grad)
    for p in range(g0, blob.shape[0]):
        t = float(blob[p])
        h = 1e-4 * max(abs(t), 1.0)
        bp, bm = blob.copy(), blob.copy()
        bp[p] = np.float32(t + h); bm[p] = np.float32(t - h)
        fd[p] = (f(bp) - f(bm)) / (float(bp[p]) - float(bm[p]))
    scale = np.abs(grad[g0:]).max()
    np.testing.assert_allclose(grad[g0:], fd[g0:], rtol=1e-5, atol=1e-6 * scale)
    assert np.count_nonzero(grad[g0:]) > 0.4 * (blob.shape[0] - g0)


def test_focal_reduces_to_bce_without_focusing():
    # gamma = 0 and no class weight: the focal loss is the plain cross-entropy
    rng = np.random.default_rng(3)
    z = rng.normal(0, 3, 40)
    yv = (rng.random(40) < 0.4).astype(np.uint8)
    Lf, df = oracle.focal(z, yv, alpha=-1.0, gamma=0.0)
    Lb, db = oracle.bce(z, yv, pos_weight=1.0)
    assert Lf == pytest.approx(Lb, rel=1e-14)
    np.testing.assert_allclose(df, db, rtol=1e-13, atol=1e-17)


def test_focal_closed_form_at_zero_logit():
    # z = 0: p = p_t = 1/2, ce = ln 2, (1 - p_t)^2 = 1/4
    L, dz = oracle.focal(np.zeros(2), np.array([1, 0]), alpha=0.25, gamma=2.0)
    ln2 = math.log(2)
    l1, l0 = 0.25 * 0.25 * ln2, 0.75 * 0.25 * ln2
    assert L == pytest.approx((l1 + l0) / 2, rel=1e-15)
    d1 = 0.25 * 0.25 * ((0.5 - 1) - 2 * 1 * 0.5 * ln2) / 2
    d0 = 0.75 * 0.25 * ((0.5 - 0) - 2 * (-1) * 0.5 * ln2) / 2
    np.testing.assert_allclose(dz, [d1, d0], rtol=1e-14)


def test_focal_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    z = rng.normal(0, 3, 60)
    yv = (rng.random(60) < 0.5).astype(np.uint8)
    for alpha, gamma in ((0.25, 2.0), (-1.0, 1.5), (0.9, 0.5)):
        _, dz = oracle.focal(z, yv, alpha, gamma)
        h = 1e-6
        # the loss is a mean of per-edge terms: differentiate edge q's term alone
        for q in range(0, 60, 7):
            lp = oracle.focal(z[q:q + 1] + h, yv[q:q + 1], alpha, gamma)[0]
            lm = oracle.focal(z[q:q + 1] - h, yv[q:q + 1], alpha, gamma)[0]
            fd = (lp - lm) / (2 * h) / z.shape[0]
            assert fd == pytest.approx(dz[q], rel=1e-6, abs=1e-13)


def test_focal_down_weights_easy_examples():
    # a confident, correct logit: the focal term is (1 - p_t)^gamma smaller than the cross-entropy
    z, yv = np.array([6.0]), np.array([1], np.uint8)
    Lf, _ = oracle.focal(z, yv, alpha=-1.0, gamma=2.0)
    Lb, _ = oracle.bce(z, yv, 1.0)
    qt = 1.0 / (1.0 + math.exp(6.0))
    assert Lf == pytest.approx(Lb * qt * qt, rel=1e-12)
