"""Pins of the oracle's interaction-network GNN (Sec. 5.2).

The main pin is a "counting network": weights chosen so that every MLP selects
one channel, which makes the edge logit a closed-form function of hit
out-degrees, in-degrees and normalised x.  The closed form is derived by hand
from the message equation and the residual node/edge updates, and it tells
apart the plausible mistakes: outgoing vs incoming sums, source vs
destination, h^k vs h^{k+1} in the edge update, the per-step weights, the
residuals and the concatenation order.
"""
import numpy as np
import pytest

import oracle
from helpers import random_graph, zero_blob
from paper_2407_12119_amd import synth

H, IT = 8, 3
C = dict(c0=0.25, c1=1 / 128, c2=-1 / 256, c3=0.5, c4=-0.75)   # exact in float32


def counting_blob(norm):
    blob, v = zero_blob(H, IT, norm=norm)
    # node encoder: h0 = (1, 0, 0, xhat0, 0...)
    W, b = v["nenc0"]; b[0] = 1; W[1, 0] = 1; b[1] = 10
    W, b = v["nenc1"]; W[0, 0] = 1; W[3, 1] = 1; b[3] = -10
    # edge encoder on [h_src | h_dst]: e0 = (1, 0, 0, xhat0(src) - xhat0(dst), 0...)
    W, b = v["eenc0"]; b[0] = 1; W[1, 3] = 1; W[1, H + 3] = -1; b[1] = 10
    W, b = v["eenc1"]; W[0, 0] = 1; W[3, 1] = 1; b[3] = -10
    for k in range(IT):
        # node net on [h | m_out | m_in]: h1 += (k+1) outdeg, h2 += 2(k+1) indeg
        W, b = v[f"node{k}_0"]; W[1, H + 0] = 1; W[2, 2 * H + 0] = 1
        W, b = v[f"node{k}_1"]; W[1, 1] = k + 1; W[2, 2] = 2 * (k + 1)
        # edge net on [e | h_src | h_dst]: e1 += h1(src), e2 += h2(dst), e5 += relu(e3)
        W, b = v[f"edge{k}_0"]; W[1, H + 1] = 1; W[2, 2 * H + 2] = 1; W[5, 3] = 1
        W, b = v[f"edge{k}_1"]; W[1, 1] = 1; W[2, 2] = 1; W[5, 5] = 1
    # classifier: z = c0 + c1 e1 + c2 e2 + c3 e3 + c4 e5
    W, b = v["cls0"]; W[0, 1] = 1; W[1, 2] = 1; W[2, 3] = 1; b[2] = 10; W[3, 5] = 1
    W, b = v["cls1"]; W[0, 0] = C["c1"]; W[0, 1] = C["c2"]; W[0, 2] = C["c3"]; W[0, 3] = C["c4"]
    b[0] = C["c0"] - 10 * C["c3"]
    return blob


def closed_form(x, src, dst, n, norm):
    outdeg = np.bincount(src, minlength=n).astype(np.float64)
    indeg = np.bincount(dst, minlength=n).astype(np.float64)
    xh = (x.astype(np.float64) - float(np.float32(norm[6]))) / float(np.float32(norm[9]))
    # h^k_1 = outdeg k(k+1)/2, h^k_2 = indeg k(k+1); the edge update at step k reads h^{k+1}
    s1 = sum(k * (k + 1) / 2 for k in range(1, IT + 1))
    s2 = sum(k * (k + 1) for k in range(1, IT + 1))
    e1 = outdeg[src] * s1
    e2 = indeg[dst] * s2
    e3 = xh[src] - xh[dst]
    e5 = IT * np.maximum(e3, 0)
    return C["c0"] + C["c1"] * e1 + C["c2"] * e2 + C["c3"] * e3 + C["c4"] * e5


@pytest.mark.parametrize("seed", range(4))
def test_counting_network_closed_form(seed):
    rng = np.random.default_rng(seed)
    n = 15
    src, dst = random_graph(n, 40, rng)
    x = rng.uniform(-30, 30, n).astype(np.float32)
    y = rng.uniform(-30, 30, n).astype(np.float32)
    z = rng.uniform(-200, 700, n).astype(np.float32)
    norm = [0, 0, 0, 1, 1, 1, 1.5, 0, 0, 12.0, 1, 1]
    blob = counting_blob(norm)
    got = oracle.gnn_forward(x, y, z, src, dst, blob, H, IT, Ce=128, D=4)
    exp = closed_form(x, src, dst, n, norm)
    np.testing.assert_allclose(got, exp, rtol=1e-12, atol=1e-12)
    # the graph really separates the readings (outdeg != indeg somewhere)
    assert (np.bincount(src, minlength=n) != np.bincount(dst, minlength=n)).any()


def test_messages_on_a_three_hit_path_by_hand():
    """0 -> 1 -> 2: outdeg = (1, 1, 0), indeg = (0, 1, 1); values worked out by hand."""
    src = np.array([0, 1], np.int32); dst = np.array([1, 2], np.int32)
    x = np.array([3.0, 1.5, -3.0], np.float32)
    y = np.zeros(3, np.float32); z = np.zeros(3, np.float32)
    norm = [0, 0, 0, 1, 1, 1, 1.5, 0, 0, 12.0, 1, 1]
    got = oracle.gnn_forward(x, y, z, src, dst, counting_blob(norm), H, IT)
    # xhat = (x - 1.5) / 12 = (0.125, 0, -0.375); s1 = 1 + 3 + 6 = 10, s2 = 2 + 6 + 12 = 20
    # edge 0->1: e1 = 1*10, e2 = indeg(1)*20 = 20, e3 = 0.125, e5 = 3*0.125
    # edge 1->2: e1 = 1*10, e2 = indeg(2)*20 = 20, e3 = 0.375, e5 = 3*0.375
    z01 = 0.25 + 10 / 128 - 20 / 256 + 0.5 * 0.125 - 0.75 * 0.375
    z12 = 0.25 + 10 / 128 - 20 / 256 + 0.5 * 0.375 - 0.75 * 1.125
    np.testing.assert_allclose(got, [z01, z12], rtol=0, atol=1e-14)


def test_relabelling_hits_permutes_logits():
    wl = synth.WORKLOADS["single_event"]
    blob = synth.init_params(synth.dataclasses.replace(wl, hidden=16, iters=2))
    rng = np.random.default_rng(4)
    n = 30
    src, dst = random_graph(n, 90, rng)
    x, y, z = (rng.uniform(-20, 20, n).astype(np.float32) for _ in range(3))
    base = oracle.gnn_forward(x, y, z, src, dst, blob, 16, 2)
    perm = rng.permutation(n)            # new index of old hit i is inv[i]
    inv = np.empty(n, np.int64); inv[perm] = np.arange(n)
    eperm = rng.permutation(src.shape[0])
    got = oracle.gnn_forward(x[perm], y[perm], z[perm], inv[src][eperm].astype(np.int32),
                             inv[dst][eperm].astype(np.int32), blob, 16, 2)
    np.testing.assert_allclose(got, base[eperm], rtol=1e-12, atol=1e-13)


def test_no_edges_gives_no_logits():
    wl = synth.WORKLOADS["single_event"]
    blob = synth.init_params(wl)
    x = np.ones(4, np.float32)
    out = oracle.gnn_forward(x, x, x, np.zeros(0, np.int32), np.zeros(0, np.int32), blob, 64, 4)
    assert out.shape == (0,)


def test_events_are_independent_in_the_batch_pipeline():
    """An event gives the same labels and logits alone and inside a batch."""
    wl = synth.WORKLOADS["batch256"]
    blob = synth.init_params(wl)
    b = synth.make_batch(wl, n_events=3, first=40)
    allr = oracle.pipeline(b, blob, 64, 4)
    one = oracle.pipeline(synth.to_batch([b.event(1)]), blob, 64, 4)
    s, e = allr["edge_offsets"][1], allr["edge_offsets"][2]
    np.testing.assert_array_equal(allr["logit"][s:e], one["logit"])
    o0, o1 = b.event_offsets[1], b.event_offsets[2]
    np.testing.assert_array_equal(allr["labels"][o0:o1], one["labels"])
