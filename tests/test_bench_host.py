"""bench.py's host-side contract, without a GPU: more than one GPU is
refused with a message, and the algorithmic work it prices the edge network
and the stages with follows the counts it documents."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr
    assert r.stdout == ""


def test_edge_network_work_counts():
    H, E, N = 64, 1000, 100
    # 2-byte states: two layers 3H -> H -> H on every edge; edge state read and
    # written, two indices, every hit state read once, outgoing sums written
    f, b = bench.edge_net_work(H, "bf16", E, N)
    assert f == 2 * (3 * H * H + H * H) * E
    assert b == (2 * H * 2 + 8) * E + H * 2 * N + 4 * H * N
    assert bench.edge_net_work(H, "bf16x2", E, N) == (f, b)
    # float32, factorised: the e segment and the second layer per edge
    f, b = bench.edge_net_work(H, "fp32", E, N)
    assert f == 2 * (H * H + H * H) * E
    assert b == (2 * H * 4 + 8) * E + 2 * H * 4 * N


def test_stage_roofline_is_max_of_compute_and_bytes():
    H, n, N, E = 64, 4, 1000, 30000
    stages = {k: (1.0, 1) for k in ("embed", "prepare", "knn", "compact", "lists", "node_enc", "edge_enc",
                                     "hit_proj", "messages", "node_net", "edge_net", "edge_cls", "components")}
    r = bench.stage_roofline(stages, 1, H, n, "bf16", N, E)
    g = r["graph"]
    assert g["flops"] == 0 and g["bytes"] == 24 * N + 16 * E
    assert abs(g["t_roof_ms"] - g["bytes"] / (bench.PEAK_HBM_GBS * 1e9) * 1e3) < 1e-4
    mp = r["message_passing"]
    # node network 3H -> H -> H per hit; edge network: the hit segments' products
    # once per hit, the edge segment and the second layer per edge; classifier
    assert mp["flops"] == n * (2 * 3 * H * H * N + 2 * H * H * N + 2 * 2 * H * H * N + 2 * H * H * E
                               + 2 * H * H * E) + 2 * (H * H + H) * E
    enc = r["encoders"]
    assert enc["flops"] == 2 * (3 * H + H * H) * N + 2 * 2 * H * H * N + 2 * H * H * E
    assert abs(r["total"]["t_ms"] - sum(v["t_ms"] for k, v in r.items() if k != "total")) < 1e-3
    for k, v in r.items():
        if k != "total":
            roof = max(v["flops"] / (bench.PEAK_TFLOPS["bf16"] * 1e12), v["bytes"] / (bench.PEAK_HBM_GBS * 1e9))
            assert abs(v["t_roof_ms"] - roof * 1e3) < 1e-4


def test_stored_tuning_is_parsed_and_checked():
    from paper_2407_12119_amd import velo
    assert bench.parse_tuning(velo, "edge_net=7, knn=5") == {"edge_net": 7, "knn": 5}
    import pytest
    for bad in ("edge_net=8", "edge_net", "nope=1", "knn=-1"):
        with pytest.raises(SystemExit):
            bench.parse_tuning(velo, bad)


def test_oracle_agreement_counts_the_edges_in_one_set_only():
    """bench.py's comparison with the oracle counts the pairs that are in one
    edge set only, by their distance class (radius band, k_max cut, other)."""
    import numpy as np
    import oracle
    from paper_2407_12119_amd import synth
    wl = synth.WORKLOADS["batch256"]
    b = synth.make_batch(wl, n_events=2, first=3)
    ref = oracle.pipeline(b, synth.centred_params(wl), wl.hidden, wl.iters, wl.radius, wl.k_max, wl.edge_logit_min)
    g = {"edge_offsets": ref["edge_offsets"].astype(np.int64), "src": ref["src"].copy(), "dst": ref["dst"].copy(),
         "logit": ref["logit"].astype(np.float32), "labels": ref["labels"].copy()}
    r = bench.oracle_agreement(synth, wl, b, ref, g)
    assert r["edges_in_one_set"] == 0 and r["jaccard"] == 1.0 and r["labels_identical"] == 1.0
    # drop an edge of event 0 from the "GPU" set: one pair in one set only
    h = dict(g, src=np.delete(g["src"], 5), dst=np.delete(g["dst"], 5), logit=np.delete(g["logit"], 5))
    h["edge_offsets"] = g["edge_offsets"].copy()
    h["edge_offsets"][1:] -= 1
    r = bench.oracle_agreement(synth, wl, b, ref, h)
    assert r["edges_in_one_set"] == 1
    assert r["of_which_within_1e-6_of_radius"] + r["of_which_at_k_max_cut"] + r["of_which_other"] == 1
