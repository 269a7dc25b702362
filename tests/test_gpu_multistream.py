"""GPU: the multi-stream throughput mode gives, batch for batch, the same
outputs as one context running the same batches one after the other (the
kernels are deterministic and every stream has its own context), and one
stream's batch matches the float64 oracle stage by stage."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                                    # noqa: E402
from paper_2407_12119_amd import multistream, synth, velo       # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_streams_match_a_single_context(precision):
    wl = synth.WORKLOADS["batch256"]
    blob = synth.centred_params(wl)
    shares = [synth.make_events(wl, 10, first=1200 + 10 * s) for s in range(3)]
    print(f"\n[case] multistream {precision} streams=3 events=30", flush=True)
    ms = multistream.MultiStream(wl, blob, precision, shares, hit_cap=6000)
    assert all(len(b) > 1 for b in ms.batches)
    for _ in range(2):                     # twice: the second pass reuses the buffers
        ms.run()
    ms.synchronize()
    ref_ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min,
                           precision, max_hits=6000, max_events=16, max_event_hits=6000)
    ref_ctx.set_params(torch.from_numpy(blob).cuda())
    for s in range(3):
        for b, h, o in zip(ms.batches[s], ms.hits[s], ms.outs[s]):
            ref = velo.graph_to_host(ref_ctx.infer(h), b.n_hits)
            got = velo.graph_to_host(o, b.n_hits)
            for k in ("labels", "edge_offsets", "src", "dst", "logit"):
                np.testing.assert_array_equal(got[k], ref[k], err_msg=f"stream {s} {k}")
    ms.close()


def test_one_stream_batch_matches_the_oracle():
    """A batch run by one of several concurrent streams (fp32), stage by stage
    against the float64 oracle: the embedding (1e-5), the rough graph rebuilt
    by the oracle from the stream context's float32 embedding (identical),
    the logits on that graph (1e-4 * max(|z|, 1)) and the labels from the
    stream's own edge decisions (identical)."""
    wl = synth.WORKLOADS["batch256"]
    blob = synth.centred_params(wl)
    shares = [synth.make_events(wl, 8, first=1300 + 8 * s) for s in range(4)]
    print("\n[case] multistream fp32 streams=4 events=32 against the oracle", flush=True)
    ms = multistream.MultiStream(wl, blob, "fp32", shares, hit_cap=5000)
    ms.run()
    ms.synchronize()
    s = 2
    batch, h, o = ms.batches[s][0], ms.hits[s][0], ms.outs[s][0]
    g = velo.graph_to_host(o, batch.n_hits)
    emb = ms.ctx[s].embed(h).cpu().numpy()
    r2 = oracle.d2max_f32(wl.radius)
    assert batch.n_events >= 2
    for b in range(batch.n_events):
        ev = batch.event(b)
        o0 = int(batch.event_offsets[b])
        e_gpu = emb[o0:o0 + ev.n]
        e_or = oracle.embed(ev.x, ev.y, ev.z, blob)
        assert np.abs(e_gpu - e_or).max() <= 1e-5 * max(1.0, np.abs(e_or).max())
        rp, col = oracle.neighbours(ev.plane, e_gpu, r2, wl.k_max)
        src, dst = oracle.csr_to_edges(rp, col)
        s0, s1 = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
        np.testing.assert_array_equal(g["src"][s0:s1], src)
        np.testing.assert_array_equal(g["dst"][s0:s1], dst)
        z = oracle.gnn_forward(ev.x, ev.y, ev.z, src, dst, blob, wl.hidden, wl.iters)
        gz = g["logit"][s0:s1]
        err = np.abs(gz - z) / np.maximum(np.abs(z), 1.0)
        assert err.size == 0 or err.max() <= 1e-4, err.max()
        lab = oracle.components(ev.n, src, dst, (gz >= wl.edge_logit_min).astype(np.uint8))
        np.testing.assert_array_equal(g["labels"][o0:o0 + ev.n], lab)
    ms.close()
