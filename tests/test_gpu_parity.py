"""GPU parity: the HIP path against the float64 oracle, stage by stage.

Each stage is compared on the GPU's own upstream outputs, so every contract
is exact or has a stated tolerance:
  * embedding: |e_gpu - e_oracle| <= 1e-5 * max(1, max |e_oracle|)
    (float32 accumulation over 128-wide layers; about 1e-6 is typical);
  * rough graph: the oracle rebuilds it from the GPU's float32 embedding with
    the same float32 distance, so the edge lists must be identical;
  * GNN logits on the GPU's graph: |z_gpu - z_oracle| <= 1e-4 * max(|z|, 1);
  * labels: the oracle's BFS on the GPU's edge decisions must give identical
    labels.
End to end (oracle from raw hits) the edge sets may differ only where the
float64 and float32 embeddings put a pair on different sides of the radius
or of the k_max cut; those are counted and bounded.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                           # noqa: E402
from paper_2407_12119_amd import synth, velo           # noqa: E402

pytestmark = pytest.mark.gpu

LOGIT_TOL = 1e-4
EMB_TOL = 1e-5


def _ctx(wl, batch, **kw):
    r2 = oracle.d2max_f32(wl.radius)
    args = dict(max_hits=max(batch.n_hits, 1), max_events=max(batch.n_events, 1),
                max_event_hits=max(batch.max_event_hits(), 1))
    args.update(kw)
    return velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, "fp32", **args)


def _setup(wl, batch, blob=None, **kw):
    print(f"\n[case] {wl.name} events={batch.n_events} hits={batch.n_hits}", flush=True)
    blob = synth.centred_params(wl) if blob is None else blob
    ctx = _ctx(wl, batch, **kw)
    ctx.set_params(torch.from_numpy(blob).cuda())
    return ctx, velo.DeviceHits.from_batch(batch), blob


def _event_edges(g, b):
    s, e = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
    return g["src"][s:e], g["dst"][s:e], g["logit"][s:e]


def _check_stages(wl, batch, blob, emb, g, events, gnn_events):
    r2 = oracle.d2max_f32(wl.radius)
    for b in events:
        ev = batch.event(b)
        o0 = int(batch.event_offsets[b])
        e_gpu = emb[o0:o0 + ev.n]
        e_or = oracle.embed(ev.x, ev.y, ev.z, blob)
        if ev.n:
            assert np.abs(e_gpu - e_or).max() <= EMB_TOL * max(1.0, np.abs(e_or).max()), f"emb event {b}"
        rp, col = oracle.neighbours(ev.plane, e_gpu, r2, wl.k_max)
        src, dst = oracle.csr_to_edges(rp, col)
        gs, gd, gz = _event_edges(g, b)
        np.testing.assert_array_equal(gs, src, err_msg=f"src event {b}")
        np.testing.assert_array_equal(gd, dst, err_msg=f"dst event {b}")
        if b in gnn_events:
            z = oracle.gnn_forward(ev.x, ev.y, ev.z, src, dst, blob, wl.hidden, wl.iters)
            err = np.abs(gz - z) / np.maximum(np.abs(z), 1.0)
            assert err.size == 0 or err.max() <= LOGIT_TOL, f"logit event {b}: {err.max()}"
        lab = oracle.components(ev.n, gs, gd, (gz >= wl.edge_logit_min).astype(np.uint8))
        np.testing.assert_array_equal(g["labels"][o0:o0 + ev.n], lab, err_msg=f"labels event {b}")


def test_single_event_all_stages():
    wl = synth.WORKLOADS["single_event"]
    batch = synth.make_batch(wl)
    ctx, hits, blob = _setup(wl, batch)
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    emb = ctx.embed(hits).cpu().numpy()
    _check_stages(wl, batch, blob, emb, g, [0], {0})
    kept = (g["logit"] >= 0).mean()
    assert 0.2 < kept < 0.8          # the bias-centred init exercises the cut


def test_staged_calls_equal_fused_call():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=6, first=10)
    ctx, hits, blob = _setup(wl, batch)
    fused = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    emb = ctx.embed(hits)
    g = ctx.build_graph(hits, emb)
    ctx.gnn(hits, g)
    ctx.components(hits, g)
    staged = velo.graph_to_host(g, batch.n_hits)
    for k in ("edge_offsets", "src", "dst", "logit", "labels"):
        np.testing.assert_array_equal(fused[k], staged[k], err_msg=k)


def test_batch_of_uneven_events_with_empty_ones():
    wl = synth.WORKLOADS["batch256"]
    evs = synth.make_events(wl, n_events=12)
    empty = synth.Event(*(np.zeros(0, dt) for dt in (np.float32, np.float32, np.float32, np.int32, np.int64, np.int32)))
    evs = [empty] + evs[:5] + [empty, empty] + evs[5:] + [empty]
    batch = synth.to_batch(evs)
    ctx, hits, blob = _setup(wl, batch)
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    emb = ctx.embed(hits).cpu().numpy()
    _check_stages(wl, batch, blob, emb, g, range(batch.n_events), {1, 2})


def test_event_alone_equals_event_in_batch():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=8, first=30)
    ctx, hits, blob = _setup(wl, batch)
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    one = synth.to_batch([batch.event(5)])
    hits1 = velo.DeviceHits.from_batch(one)
    g1 = velo.graph_to_host(ctx.infer(hits1), one.n_hits)
    s, e = _event_edges(g, 5)[0], None
    gs, gd, gz = _event_edges(g, 5)
    np.testing.assert_array_equal(gs, g1["src"])
    np.testing.assert_array_equal(gd, g1["dst"])
    np.testing.assert_array_equal(gz, g1["logit"])
    o0 = int(batch.event_offsets[5])
    np.testing.assert_array_equal(g["labels"][o0:o0 + one.n_hits], g1["labels"])


def test_runs_are_bitwise_deterministic():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=16)
    ctx, hits, _ = _setup(wl, batch)
    a = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    b = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    for k in ("edge_offsets", "src", "dst", "logit", "labels"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_end_to_end_against_oracle_from_raw_hits():
    """Full oracle from raw hits: differences only in radius/k bands."""
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=2, first=3)
    ctx, hits, blob = _setup(wl, batch)
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    ref = oracle.pipeline(batch, blob, wl.hidden, wl.iters, wl.radius, wl.k_max)
    r2 = oracle.d2max_f32(wl.radius)
    for b in range(batch.n_events):
        gs, gd, gz = _event_edges(g, b)
        s, e = int(ref["edge_offsets"][b]), int(ref["edge_offsets"][b + 1])
        o0 = int(batch.event_offsets[b])
        eo = ref["emb"][o0:o0 + int(np.diff(batch.event_offsets)[b])]
        A = set(zip(gs.tolist(), gd.tolist()))
        Bs = set(zip(ref["src"][s:e].tolist(), ref["dst"][s:e].tolist()))
        diff = A ^ Bs
        # each differing pair must sit within 1e-5 relative of the radius or of its row's k-th distance;
        # pairs within 1e-6 relative of the radius itself are reported separately
        near_r = at_k = 0
        for (i, j) in diff:
            d2 = float(((eo[i] - eo[j]) ** 2).sum())
            row = [jj for (ii, jj) in Bs if ii == i]
            dk = max(((eo[i] - eo[jj]) ** 2).sum() for jj in row) if row else r2
            assert abs(d2 - r2) <= 1e-5 * r2 or abs(d2 - dk) <= 1e-5 * max(dk, 1e-12), (b, i, j)
            if abs(np.sqrt(d2) - wl.radius) <= 1e-6 * wl.radius:
                near_r += 1
            elif abs(d2 - dk) <= 1e-5 * max(dk, 1e-12):
                at_k += 1
        print(f"  event {b}: {len(Bs)} oracle edges, {len(diff)} differ: {near_r} within 1e-6 of the "
              f"radius, {at_k} at the k_max cut, {len(diff) - near_r - at_k} within 1e-5 of the radius",
              flush=True)
        assert len(diff) <= 0.001 * max(len(Bs), 1) + 2


def test_capacity_overflow_is_reported():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=2)
    ctx, hits, _ = _setup(wl, batch)
    out = ctx.alloc_outputs(hits, edge_capacity=100)
    with pytest.raises(velo.VeloError) as ei:
        ctx.infer(hits, out)
    assert ei.value.status == velo.VELO_ERR_CAPACITY
    assert int(out["n_edges"].cpu()[0]) > 100
    # the context recovers: a call with room succeeds
    ctx.infer(hits)


def test_invalid_hits_are_reported():
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=2)
    ctx, hits, _ = _setup(wl, batch)
    bad = velo.DeviceHits.from_batch(batch)
    bad.plane = bad.plane.flip(0).contiguous()          # not sorted by plane
    with pytest.raises(velo.VeloError) as ei:
        ctx.infer(bad)
    assert ei.value.status == velo.VELO_ERR_INPUT
    bad2 = velo.DeviceHits.from_batch(batch)
    bad2.x[3] = float("nan")
    with pytest.raises(velo.VeloError) as ei:
        ctx.infer(bad2)
    assert ei.value.status == velo.VELO_ERR_INPUT
    bad3 = velo.DeviceHits.from_batch(batch)
    bad3.plane[0] = 26
    with pytest.raises(velo.VeloError):
        ctx.infer(bad3)
    ctx.infer(hits)


def test_given_graph_must_be_grouped_by_source():
    """velo_gnn takes a graph whose edges come grouped by source within each
    event (as velo_build_graph writes it); another order is an input error,
    and the context works afterwards."""
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=2, first=3)
    ctx, hits, _ = _setup(wl, batch)
    g = ctx.build_graph(hits, ctx.embed(hits))
    n0 = int(g["edge_offsets"][1].cpu())
    assert n0 > 2
    bad = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in g.items()}
    bad["edge_src"][:n0] = bad["edge_src"][:n0].flip(0)
    bad["edge_dst"][:n0] = bad["edge_dst"][:n0].flip(0)
    with pytest.raises(velo.VeloError) as ei:
        ctx.gnn(hits, bad)
    assert ei.value.status == velo.VELO_ERR_INPUT
    ctx.gnn(hits, g)


def test_given_graph_with_a_negative_interior_edge_offset():
    """A caller's edge_offsets with a negative entry for an event other than
    the first (e.g. [0, -5, n, E]) is an input error caught by every event's
    own window check, before any edge index is formed; the context works
    afterwards."""
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=3, first=3)
    ctx, hits, _ = _setup(wl, batch)
    g = ctx.build_graph(hits, ctx.embed(hits))
    for bad_off in (-5, -(1 << 30)):
        bad = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in g.items()}
        bad["edge_offsets"][1] = bad_off
        with pytest.raises(velo.VeloError) as ei:
            ctx.gnn(hits, bad)
        assert ei.value.status == velo.VELO_ERR_INPUT
        with pytest.raises(velo.VeloError) as ei:
            ctx.components(hits, bad)
        assert ei.value.status == velo.VELO_ERR_INPUT
    z = ctx.gnn(hits, g)
    assert z is not None


def _hub_event(rng, counts):
    """Hits on a few planes with the given counts; an event plus a given graph
    whose destinations are skewed onto 20 hub hits per plane."""
    plane = np.repeat(np.arange(len(counts)), counts).astype(np.int32)
    n = plane.size
    r = np.sqrt(rng.uniform(5.1 ** 2, 42.0 ** 2, n))
    phi = rng.uniform(0, 2 * np.pi, n)
    ev = synth.Event((r * np.cos(phi)).astype(np.float32), (r * np.sin(phi)).astype(np.float32),
                     synth.PLANE_Z[plane].astype(np.float32), plane, np.full(n, -1, np.int64),
                     np.full(n, -1, np.int32))
    po = np.concatenate([[0], np.cumsum(counts)])
    src, dst = [], []
    for i in range(n):
        p = plane[i]
        targets = []
        for dp in (1, 2):
            if p + dp < len(counts) and counts[p + dp] > 0:
                lo, hi = po[p + dp], po[p + dp + 1]
                hubs = np.arange(lo, min(lo + 20, hi))
                k = int(rng.integers(1, 9))
                pick = np.where(rng.random(k) < 0.5, rng.choice(hubs, k), rng.integers(lo, hi, k))
                targets.extend(np.unique(pick).tolist())
        for j in sorted(set(targets)):
            src.append(i)
            dst.append(j)
    return ev, np.array(src, np.int32), np.array(dst, np.int32)


def test_incoming_lists_of_large_planes_and_hubs():
    """Incoming lists on a plane of more hits than one LDS slice holds (2,048)
    and on hub hits with hundreds of incoming edges: the GNN on this given
    graph must match the oracle's logits."""
    wl = synth.WORKLOADS["batch256"]
    rng = np.random.default_rng(2407)
    ev, src, dst = _hub_event(rng, [0, 0, 0, 300, 300, 2600, 300, 200])
    indeg = np.bincount(dst, minlength=ev.n)
    assert indeg.max() > 128
    batch = synth.to_batch([ev])
    ctx, hits, blob = _setup(wl, batch, max_edges=max(len(src), 1))
    out = ctx.alloc_outputs(hits, edge_capacity=len(src))
    out["edge_src"][:len(src)] = torch.from_numpy(src).cuda()
    out["edge_dst"][:len(dst)] = torch.from_numpy(dst).cuda()
    out["edge_offsets"].copy_(torch.tensor([0, len(src)], dtype=torch.int32))
    out["n_edges"].fill_(len(src))
    ctx.gnn(hits, out)
    gz = out["edge_logit"][:len(src)].cpu().numpy()
    z = oracle.gnn_forward(ev.x, ev.y, ev.z, src, dst, blob, wl.hidden, wl.iters)
    err = np.abs(gz - z) / np.maximum(np.abs(z), 1.0)
    assert err.max() <= LOGIT_TOL, err.max()


def test_zero_events_and_all_empty_events():
    wl = synth.WORKLOADS["batch256"]
    empty = synth.Event(*(np.zeros(0, dt) for dt in (np.float32, np.float32, np.float32, np.int32, np.int64, np.int32)))
    batch = synth.to_batch([empty, empty, empty])
    ctx, hits, _ = _setup(wl, batch, max_hits=16, max_events=4, max_event_hits=16)
    g = velo.graph_to_host(ctx.infer(hits), 0)
    assert g["n_edges"] == 0 and g["edge_offsets"].tolist() == [0, 0, 0, 0]
    z = synth.to_batch([])
    hz = velo.DeviceHits.from_batch(z)
    out = ctx.infer(hz)
    assert int(out["n_edges"].cpu()[0]) == 0


def test_k_max_saturation_and_single_plane_pairs():
    """A dense cluster: every hit sees more than k_max candidates; ties by index."""
    wl = synth.dataclasses.replace(synth.WORKLOADS["batch256"], k_max=4)
    rng = np.random.default_rng(7)
    n = 120
    plane = np.sort(rng.integers(0, 4, n)).astype(np.int32)
    x = rng.normal(10, 0.001, n).astype(np.float32)
    y = rng.normal(10, 0.001, n).astype(np.float32)
    z = synth.PLANE_Z[plane].astype(np.float32)
    ev = synth.Event(x, y, z, plane, np.zeros(n, np.int64), np.full(n, -1, np.int32))
    batch = synth.to_batch([ev])
    blob = synth.centred_params(synth.WORKLOADS["batch256"])
    ctx, hits, blob = _setup(wl, batch, blob=blob)
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    emb = ctx.embed(hits).cpu().numpy()
    _check_stages(wl, batch, blob, emb, g, [0], {0})
    assert np.bincount(g["src"], minlength=n).max() == 4


@pytest.mark.parametrize("k_max", [32, 5])
def test_exactly_tied_distances_cut_at_k_max(k_max):
    """Hits on a coarse grid: many candidates share the same embedding, so
    distances tie exactly and the k_max-th one usually ties with dropped
    ones; the lowest candidate indices must win, as in the oracle (Sec. 5.1
    keeps the k_max nearest; ties go by index)."""
    wl = synth.dataclasses.replace(synth.WORKLOADS["batch256"], k_max=k_max)
    rng = np.random.default_rng(11)
    n = 400
    plane = np.sort(rng.integers(0, 6, n)).astype(np.int32)
    x = (10 + 0.002 * rng.integers(0, 3, n)).astype(np.float32)
    y = (10 + 0.002 * rng.integers(0, 2, n)).astype(np.float32)
    z = synth.PLANE_Z[plane].astype(np.float32)
    ev = synth.Event(x, y, z, plane, np.zeros(n, np.int64), np.full(n, -1, np.int32))
    batch = synth.to_batch([ev])
    ctx, hits, blob = _setup(wl, batch)
    emb = ctx.embed(hits)
    g = velo.graph_to_host(ctx.build_graph(hits, emb), batch.n_hits)
    e32 = emb.cpu().numpy()
    rp, col = oracle.neighbours(ev.plane, e32, oracle.d2max_f32(wl.radius), wl.k_max)
    deg = np.diff(rp)
    full_rp, _ = oracle.neighbours(ev.plane, e32, oracle.d2max_f32(wl.radius), n)
    assert (np.diff(full_rp) > k_max).mean() > 0.5          # the cut is active for most hits
    src, dst = oracle.csr_to_edges(rp, col)
    np.testing.assert_array_equal(g["src"], src)
    np.testing.assert_array_equal(g["dst"], dst)
    assert deg.max() == k_max


def test_dense_event_candidate_windows_beyond_lds():
    """One event of ~17k hits whose plane windows hold up to ~2,200
    candidates: windows above the LDS staging size are read through L2 and
    must give the oracle's graph exactly, like the staged ones."""
    wl = synth.WORKLOADS["batch256"]
    ev = synth.make_event(synth.EventRecipe(1500, 1.0, 1500.0, 0.05), synth.event_rng(77, 0))
    counts = np.bincount(ev.plane, minlength=synth.N_PLANES)
    window = counts[1:] + np.concatenate([counts[2:], [0]])
    assert window.max() > 1024 and window.min() < 1024
    batch = synth.to_batch([ev])
    ctx, hits, blob = _setup(wl, batch)
    emb = ctx.embed(hits)
    g = velo.graph_to_host(ctx.build_graph(hits, emb), batch.n_hits)
    rp, col = oracle.neighbours(ev.plane, emb.cpu().numpy(), oracle.d2max_f32(wl.radius), wl.k_max)
    src, dst = oracle.csr_to_edges(rp, col)
    np.testing.assert_array_equal(g["src"], src)
    np.testing.assert_array_equal(g["dst"], dst)


@pytest.mark.slow
def test_full_batch256_sampled():
    """The 256-event workload in the benchmark's launch configuration: every
    event's rough graph and labels exactly, logits of sampled events."""
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl)
    ctx, hits, blob = _setup(wl, batch)
    g = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    emb = ctx.embed(hits).cpu().numpy()
    sizes = np.diff(batch.event_offsets)
    big = int(np.argmax(sizes))
    _check_stages(wl, batch, blob, emb, g, range(batch.n_events), {0, big})


def test_captured_graph_replays_match_eager_calls():
    """velo_infer captured once and replayed: every replay (with eager work and
    synchronisations between them, and new hits written into the same buffers)
    equals the eager result."""
    wl = synth.WORKLOADS["batch256"]
    b1 = synth.make_batch(wl, n_events=6, first=100)
    side = torch.cuda.Stream()
    torch.cuda.set_stream(side)          # capture needs a stream other than the legacy default one
    ctx, hits, blob = _setup(wl, b1)
    out = ctx.alloc_outputs(hits)
    graph = ctx.capture(hits, out)
    eager = velo.graph_to_host(ctx.infer(hits), b1.n_hits)
    for rep in range(3):
        for k in ("edge_logit", "labels", "edge_src"):
            out[k].fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        ctx.check()
        got = velo.graph_to_host(out, b1.n_hits)
        for k in ("edge_offsets", "src", "dst", "logit", "labels"):
            np.testing.assert_array_equal(got[k], eager[k], err_msg=f"replay {rep} {k}")
        ctx.infer(hits)                      # eager work between replays
        torch.cuda.synchronize()
    # new events of the same total size written into the captured buffers
    b2 = synth.to_batch([b1.event(b) for b in reversed(range(b1.n_events))])
    for name, arr in (("event_offsets", b2.event_offsets), ("x", b2.x), ("y", b2.y), ("z", b2.z),
                      ("plane", b2.plane)):
        getattr(hits, name).copy_(torch.from_numpy(arr))
    graph.launch()
    torch.cuda.synchronize()
    ctx.check()
    got = velo.graph_to_host(out, b2.n_hits)
    ref = velo.graph_to_host(ctx.infer(velo.DeviceHits.from_batch(b2)), b2.n_hits)
    for k in ("edge_offsets", "src", "dst", "logit", "labels"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    graph.close()
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream())


@pytest.mark.parametrize("kind", ["empty_and_tiny", "one_hit_per_plane"])
def test_xcd_work_walk_on_degenerate_batches(kind):
    """H = 128 with the 16-wavefront edge MLPs and their per-XCD work walk
    (candidate 7) on batches with empty events, one-hit events and hits
    without out-edges: bitwise the results of the default launches."""
    wl = synth.WORKLOADS["batch1000_h128"]
    empty = synth.Event(*(np.zeros(0, dt) for dt in (np.float32, np.float32, np.float32, np.int32, np.int64,
                                                      np.int32)))
    if kind == "empty_and_tiny":
        evs = [empty, synth.make_batch(wl, n_events=1, first=3).event(0), empty, empty]
        one = synth.make_batch(wl, n_events=1, first=4).event(0)
        k = np.arange(1)
        evs.append(synth.Event(one.x[k], one.y[k], one.z[k], one.plane[k], one.pid[k], one.next_hit[k] * 0 - 1))
        evs.append(empty)
    else:
        # one hit on each plane: every hit has at most two out-edges
        plane = np.arange(26, dtype=np.int32)
        evs = [synth.Event(np.full(26, 10.0, np.float32), np.full(26, 10.0, np.float32),
                           synth.PLANE_Z[plane].astype(np.float32), plane, np.zeros(26, np.int64),
                           np.full(26, -1, np.int32))]
    batch = synth.to_batch(evs)
    print(f"\n[case] xcd work walk {kind} events={batch.n_events} hits={batch.n_hits}", flush=True)
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, "bf16",
                       max_hits=max(batch.n_hits, 1), max_events=batch.n_events,
                       max_event_hits=max(batch.max_event_hits(), 1))
    ctx.set_params(torch.from_numpy(synth.centred_params(wl)).cuda())
    hits = velo.DeviceHits.from_batch(batch)
    ref = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    ctx.set_tuning(7)
    got = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    for k in ("edge_offsets", "src", "dst", "logit", "labels"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    print(f"  {ref['n_edges']} edges identical", flush=True)


def test_captured_graph_replays_with_the_xcd_work_counters():
    """H = 128 with the 16-wavefront edge MLPs (candidate 7): their per-XCD
    work counters are cleared by a fill kernel before every launch, which a
    captured graph replays too.  Every replay, with eager calls in between,
    equals the eager result bitwise."""
    wl = synth.WORKLOADS["batch1000_h128"]
    batch = synth.make_batch(wl, n_events=5, first=7)
    print(f"\n[case] graph replays H=128 bf16 candidate 7 events={batch.n_events} hits={batch.n_hits}", flush=True)
    side = torch.cuda.Stream()
    torch.cuda.set_stream(side)
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, "bf16",
                       max_hits=batch.n_hits, max_events=batch.n_events, max_event_hits=batch.max_event_hits())
    ctx.set_params(torch.from_numpy(synth.centred_params(wl)).cuda())
    ctx.set_tuning(7)
    hits = velo.DeviceHits.from_batch(batch)
    out = ctx.alloc_outputs(hits)
    graph = ctx.capture(hits, out)
    eager = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    for rep in range(3):
        for k in ("edge_logit", "labels"):
            out[k].fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        ctx.check()
        got = velo.graph_to_host(out, batch.n_hits)
        for k in ("edge_offsets", "src", "dst", "logit", "labels"):
            np.testing.assert_array_equal(got[k], eager[k], err_msg=f"replay {rep} {k}")
        ctx.infer(hits)
        torch.cuda.synchronize()
    graph.close()
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream())
    print(f"  {eager['n_edges']} edges, 3 replays identical", flush=True)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_autotuned_launches_give_identical_results(precision):
    """Launch parameters and tile shapes (blocks per CU, MLP workgroup size,
    k-NN query run length, XCD-blocked work mapping) change only which wave
    processes which unit: outputs are bitwise those of the default launches,
    for every candidate of the autotuner's table and for its pick."""
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=24, first=40)
    print(f"\n[case] autotune {precision} events={batch.n_events} hits={batch.n_hits}", flush=True)
    r2 = oracle.d2max_f32(wl.radius)
    ctx = velo.Context(wl.hidden, wl.iters, r2, wl.k_max, wl.edge_logit_min, precision,
                       max_hits=batch.n_hits, max_events=batch.n_events, max_event_hits=batch.max_event_hits())
    ctx.set_params(torch.from_numpy(synth.centred_params(wl)).cuda())
    hits = velo.DeviceHits.from_batch(batch)
    if precision == "fp8":
        ctx.calibrate(hits)          # fixed scales for every candidate
    ref = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    for cand in range(len(velo.AUTOTUNE_CANDIDATES)):
        ctx.set_tuning(cand)
        got = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
        for k in ("edge_offsets", "src", "dst", "logit", "labels"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"candidate {cand}: {k}")
    ctx.set_tuning(None)
    out = ctx.alloc_outputs(hits)
    choice = ctx.autotune(hits, out)
    print(f"  choice {choice}", flush=True)
    got = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    for k in ("edge_offsets", "src", "dst", "logit", "labels"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    with pytest.raises(velo.VeloError):
        ctx.set_tuning(len(velo.AUTOTUNE_CANDIDATES))


@pytest.mark.parametrize("precision", ["bf16", "bf16x2", "fp8"])
def test_tile_shapes_at_width_128_give_identical_results(precision):
    """H = 128: every candidate of the autotuner's table, including the
    16-wavefront workgroups of the edge MLPs (one chunk per wavefront, half a
    K block of weight fragments at a time), gives bitwise the default
    results."""
    wl = synth.WORKLOADS["batch1000_h128"]
    batch = synth.make_batch(wl, n_events=5, first=11)
    print(f"\n[case] tile shapes H=128 {precision} events={batch.n_events} hits={batch.n_hits}", flush=True)
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, precision,
                       max_hits=batch.n_hits, max_events=batch.n_events, max_event_hits=batch.max_event_hits())
    ctx.set_params(torch.from_numpy(synth.centred_params(wl)).cuda())
    hits = velo.DeviceHits.from_batch(batch)
    if precision == "fp8":
        ctx.calibrate(hits)          # fixed scales for every candidate
    ref = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
    for cand in range(len(velo.AUTOTUNE_CANDIDATES)):
        ctx.set_tuning(cand)
        got = velo.graph_to_host(ctx.infer(hits), batch.n_hits)
        for k in ("edge_offsets", "src", "dst", "logit", "labels"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"candidate {cand}: {k}")
    print(f"  {ref['n_edges']} edges, {len(velo.AUTOTUNE_CANDIDATES)} candidates identical", flush=True)


def test_plane_sweep_variant_matches_oracle_sweep():
    """The paper's two plane sweeps (Sec. 7.3), kept as a comparison variant:
    labels bit-exact against the oracle's sweep on the GPU's own decisions,
    and the share of hits they label differently from exact components."""
    wl = synth.WORKLOADS["batch256"]
    batch = synth.make_batch(wl, n_events=6, first=60)
    ctx, hits, blob = _setup(wl, batch)
    out = ctx.infer(hits)
    exact = out["labels"].clone()
    ctx.components_sweep(hits, out)
    g = velo.graph_to_host(out, batch.n_hits)
    sweep = g["labels"]
    ex = exact.cpu().numpy()
    differ = 0
    for b in range(batch.n_events):
        ev = batch.event(b)
        o = int(batch.event_offsets[b])
        s, e = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
        keep = (g["logit"][s:e] >= wl.edge_logit_min).astype(np.uint8)
        ref = oracle.components_sweep(ev.plane, g["src"][s:e], g["dst"][s:e], keep)
        np.testing.assert_array_equal(sweep[o:o + ev.n], ref, err_msg=f"event {b}")
        np.testing.assert_array_equal(ex[o:o + ev.n], oracle.components(ev.n, g["src"][s:e], g["dst"][s:e], keep))
        differ += int(np.sum(ref != ex[o:o + ev.n]))
    print(f"[sweep] hits labelled differently from exact components: {differ} of {batch.n_hits}", flush=True)
    assert differ > 0          # the centred init keeps branching graphs, where the sweep is not exact


def test_plane_sweep_variant_on_the_worked_counterexample():
    """Hits sorted by plane: 0, 1 on plane 0 and 2, 3 on plane 1; kept edges
    0->2, 1->2, 1->3.  The sweeps give [0, 0, 0, 1]; the component is {0..3}."""
    wl = synth.WORKLOADS["batch256"]
    plane = np.array([0, 0, 1, 1], np.int32)
    x = np.array([10.0, 11.0, 10.0, 11.0], np.float32)
    ev = synth.Event(x, x.copy(), synth.PLANE_Z[plane].astype(np.float32), plane, np.full(4, -1, np.int64),
                     np.full(4, -1, np.int32))
    batch = synth.to_batch([ev])
    ctx, hits, _ = _setup(wl, batch)
    out = ctx.alloc_outputs(hits)
    out["edge_offsets"].copy_(torch.tensor([0, 3], dtype=torch.int32))
    out["edge_src"][:3].copy_(torch.tensor([0, 1, 1], dtype=torch.int32))
    out["edge_dst"][:3].copy_(torch.tensor([2, 2, 3], dtype=torch.int32))
    out["edge_logit"][:3].fill_(1.0)
    out["n_edges"].fill_(3)
    ctx.components_sweep(hits, out)
    assert out["labels"].cpu().numpy().tolist() == [0, 0, 0, 1]
    ctx.components(hits, out)
    assert out["labels"].cpu().numpy().tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("kind", ["batch", "ties", "dense"])
def test_paper_neighbour_loop_variant_gives_the_same_graph(kind):
    """The paper's per-hit neighbour loop (Sec. 7.2), kept as a comparison
    variant, selects the same k_max nearest under (d2, index) as the
    wavefront search: identical graphs, including exact ties and windows of
    more than 512 candidates."""
    wl = synth.WORKLOADS["batch256"]
    if kind == "batch":
        batch = synth.make_batch(wl, n_events=8, first=70)
    elif kind == "ties":
        rng = np.random.default_rng(11)
        n = 400
        plane = np.sort(rng.integers(0, 6, n)).astype(np.int32)
        x = (10 + 0.002 * rng.integers(0, 3, n)).astype(np.float32)
        y = (10 + 0.002 * rng.integers(0, 2, n)).astype(np.float32)
        batch = synth.to_batch([synth.Event(x, y, synth.PLANE_Z[plane].astype(np.float32), plane,
                                            np.zeros(n, np.int64), np.full(n, -1, np.int32))])
    else:
        batch = synth.to_batch([synth.make_event(synth.EventRecipe(1500, 1.0, 1500.0, 0.05),
                                                 synth.event_rng(77, 0))])
    ctx, hits, _ = _setup(wl, batch)
    emb = ctx.embed(hits)
    a = velo.graph_to_host(ctx.build_graph(hits, emb), batch.n_hits)
    b = velo.graph_to_host(ctx.build_graph_loop(hits, emb), batch.n_hits)
    for k in ("edge_offsets", "src", "dst"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    # and the oracle's neighbour sets on the same float32 embedding
    e_host = emb.cpu().numpy()
    r2 = oracle.d2max_f32(wl.radius)
    for ev_i in range(batch.n_events):
        ev = batch.event(ev_i)
        o0 = int(batch.event_offsets[ev_i])
        rp, col = oracle.neighbours(ev.plane, e_host[o0:o0 + ev.n], r2, wl.k_max)
        src, dst = oracle.csr_to_edges(rp, col)
        s0, s1 = int(b["edge_offsets"][ev_i]), int(b["edge_offsets"][ev_i + 1])
        np.testing.assert_array_equal(b["src"][s0:s1], src, err_msg=f"loop src event {ev_i}")
        np.testing.assert_array_equal(b["dst"][s0:s1], dst, err_msg=f"loop dst event {ev_i}")
