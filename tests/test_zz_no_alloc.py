"""GPU: velo_components_noalloc (no context, no device allocation) against
velo_components on the same scored graphs, two calls in a row with the
second batch smaller, plus the refusals and a recovery after invalid input.
Labels are integers: bit-exact."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                           # noqa: E402
from paper_2407_12119_amd import synth, velo           # noqa: E402

pytestmark = pytest.mark.gpu


def _scored_graph(wl, batch, blob):
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, "fp32",
                       max_hits=batch.n_hits, max_events=batch.n_events, max_event_hits=batch.max_event_hits())
    ctx.set_params(torch.from_numpy(blob).cuda())
    hits = velo.DeviceHits.from_batch(batch)
    out = ctx.infer(hits)
    ctx.components(hits, out)        # the existing entry point's labels
    return ctx, hits, out


def test_noalloc_components_match_the_context_entry_point_on_two_calls():
    wl = synth.WORKLOADS["batch256"]
    blob = synth.centred_params(wl)
    big = synth.make_batch(wl, n_events=12, first=30)
    small = synth.make_batch(wl, n_events=3, first=90)
    assert small.n_hits < big.n_hits
    for batch in (big, small):
        print(f"\n[case] noalloc events={batch.n_events} hits={batch.n_hits}", flush=True)
        ctx, hits, out = _scored_graph(wl, batch, blob)
        ref = out["labels"][:batch.n_hits].clone()
        out["labels"].fill_(-7)
        velo.components_noalloc(hits, out, wl.edge_logit_min, batch.max_event_hits())
        got = out["labels"][:batch.n_hits]
        assert torch.equal(got, ref)
        # and the oracle's components on the same decisions, for one event
        g = velo.graph_to_host(out, batch.n_hits)
        b = batch.n_events - 1
        s, e = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
        o0, o1 = int(batch.event_offsets[b]), int(batch.event_offsets[b + 1])
        lab = oracle.components(o1 - o0, g["src"][s:e], g["dst"][s:e], (g["logit"][s:e] >= 0).astype(np.uint8))
        np.testing.assert_array_equal(g["labels"][o0:o1], lab)
        kept = int((g["logit"] >= 0).sum())
        print(f"  {g['n_edges']} edges, {kept} kept, {len(np.unique(g['labels']))} labels: identical", flush=True)
        ctx.close()


def test_noalloc_components_refusals_and_recovery():
    wl = synth.WORKLOADS["batch256"]
    blob = synth.centred_params(wl)
    batch = synth.make_batch(wl, n_events=2, first=7)
    ctx, hits, out = _scored_graph(wl, batch, blob)
    ref = out["labels"][:batch.n_hits].clone()
    # refused on the host before any launch: sizes beyond the fixed working memory
    for h, mx in ((velo.DeviceHits(hits.event_offsets, hits.x, hits.y, hits.z, hits.plane, hits.n_events,
                                   (1 << 20) + 1, hits.max_event_hits), batch.max_event_hits()),
                  (hits, 1 << 17)):
        with pytest.raises(velo.VeloError) as ei:
            velo.components_noalloc(h, out, wl.edge_logit_min, mx)
        assert ei.value.status == velo.VELO_ERR_CAPACITY
    # an event larger than max_event_hits is invalid input (device validation)
    with pytest.raises(velo.VeloError) as ei:
        velo.components_noalloc(hits, out, wl.edge_logit_min, batch.max_event_hits() - 1)
    assert ei.value.status == velo.VELO_ERR_INPUT
    # an edge index outside its event: invalid input; the next valid call is unaffected
    bad = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in out.items()}
    bad["edge_dst"][3] = 1 << 24
    with pytest.raises(velo.VeloError) as ei:
        velo.components_noalloc(hits, bad, wl.edge_logit_min, batch.max_event_hits())
    assert ei.value.status == velo.VELO_ERR_INPUT
    out["labels"].fill_(-7)
    velo.components_noalloc(hits, out, wl.edge_logit_min, batch.max_event_hits())
    assert torch.equal(out["labels"][:batch.n_hits], ref)
    ctx.close()
